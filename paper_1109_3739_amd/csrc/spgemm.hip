// SpGEMM C = A*B over a semiring on one gfx950 GPU.
//
// What is computed is the column-wise product of Section 3 (Algorithm 1):
// column j of C is the semiring sum, over the nonzeros B(k,j), of
// A(:,k) "times" B(k,j).  The paper's local kernel (HyperSparseGEMM, an
// outer product merged through a priority queue, Section 3.1) is prior art
// for a serial CPU; here every output column is formed independently by a
// wave or a workgroup, and the only property kept from the paper's kernel
// is that no pass is proportional to a matrix dimension when the operands
// are hypersparse (DCSC operands are iterated over their nonempty columns;
// the column lookup into a DCSC A uses the AUX index of Section 3.2).
//
// Two phases.
//   plan (symbolic): per-entry lookup of A's columns, per-column number of
//     multiplications, binning of the columns by that count, exact output
//     counts (a wave-wide sort for tiny columns, an LDS hash for medium ones,
//     an LDS bitmap over the row space for heavy ones, which also yields
//     per-row-block counts), int64 scan into column pointers, and a list of
//     row-range "parts" (each fits one workgroup's LDS) for the numeric phase.
//   exec (numeric): tiny columns are re-formed by their wave and written;
//     every part is accumulated in LDS either through a bitmap over its row
//     range (rank of a row = popcount prefix, which also yields sorted
//     output) or through a hash table followed by an LDS bitonic sort.
#include <algorithm>
#include <cstring>
#include <memory>

#include "common.h"
#include "operand.h"
#include "plan.h"
#include "scan.h"

namespace spx {

// Semiring for the boolean (pattern only) case; values are never touched.
template <typename T>
struct Semiring<SPX_OR_AND, T> {
  static constexpr bool kUsesA = false, kUsesB = false;
  __device__ static T mul(T a, T) { return a; }
  __device__ static T add(T acc, T) { return acc; }
  __device__ static T ident() { return T(0); }
  __device__ static void lds_acc(T*, T) {}
};

// ------------------------------------------------------------------ bins
// Columns (slots of B) are binned by their number of multiplications mu.
// The bin id is also the processing order: heavy columns first.
//   0 .. 40   bitmap-counted columns, id = 40 - floor(log2 mu)
//   41 .. 48  hash-counted columns, table of 2^(15 - (id - 41)) keys
//   49        tiny columns (mu <= tiny_max, at most 64): one wave each
//   50        columns without products
constexpr int kBinHash0 = 41;
constexpr int kBinTiny = 49;
constexpr int kBinEmpty = 50;
constexpr int kNumBins = 51;
constexpr int kHashLog2Max = 15;
constexpr int kHashLog2Min = 8;
constexpr int kBitmapChunkLog2 = 20;                          // rows per bitmap-count chunk
constexpr int32_t kSplitMin = 32;  // A columns longer than this get a split-table row

__device__ __forceinline__ int floor_log2_u64(uint64_t x) { return 63 - __clzll(x); }
__device__ __forceinline__ int ceil_log2_u64(uint64_t x) { return x <= 1 ? 0 : 64 - __clzll(x - 1); }

struct BinCfg {
  int64_t tiny_max, hash_max;
};

__device__ __forceinline__ int bin_of(int64_t mu, const BinCfg& c) {
  if (mu <= 0) return kBinEmpty;
  if (mu <= c.tiny_max) return kBinTiny;
  if (mu <= c.hash_max) {
    int s = ceil_log2_u64((uint64_t)mu) + 1;
    if (s < kHashLog2Min) s = kHashLog2Min;
    return kBinHash0 + (kHashLog2Max - s);
  }
  int id = 40 - floor_log2_u64((uint64_t)mu);
  return id < 0 ? 0 : id;
}

// ------------------------------------------------------------------ kernels: setup
// For every stored B(k,j): where column k of A starts, how long it is, and
// its row of the split table (-1 for short columns).
__global__ void k_rowinfo(Operand A, Operand B, const int64_t* aux, int64_t chunk, const int64_t* sid_off,
                          int64_t* bq_a0, int32_t* bq_alen, int32_t* bq_split, unsigned* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < B.nnz; q += stride) {
    const int32_t k = B.ir[q];
    int64_t a0 = 0, a1 = 0, slot = -1;
    if (k < 0 || k >= A.n) {
      atomicOr(err, 1u);
    } else {
      slot = column_slot(A, aux, chunk, k);
      if (slot >= 0) {
        a0 = load_ptr(A.cp, A.ptr_t, slot);
        a1 = load_ptr(A.cp, A.ptr_t, slot + 1);
      }
    }
    bq_a0[q] = a0;
    bq_alen[q] = (int32_t)(a1 - a0);
    bq_split[q] = (sid_off && a1 - a0 > kSplitMin) ? (int32_t)sid_off[slot] : -1;
  }
}

// Split table of the long columns of A (see ProdSrc).
struct LongColumn {
  Operand A;
  __device__ int64_t operator()(int64_t k) const { return slot_begin(A, k + 1) - slot_begin(A, k) > kSplitMin; }
};

__global__ void k_split_rows(Operand A, int64_t nslots, const int64_t* sid_off, int32_t* slot_of_split) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nslots; k += (int64_t)gridDim.x * blockDim.x)
    if (slot_begin(A, k + 1) - slot_begin(A, k) > kSplitMin) slot_of_split[sid_off[k]] = (int32_t)k;
}

// Row of the split table of one long column: entry b (< sstride - 1) is the
// first position whose row lies in row block b or later, the last entry the
// column length.  One wave per column walks its rows once: the entry at
// position e fills the blocks after its predecessor's block up to its own.
__global__ void k_split_fill(Operand A, const int64_t* nsplit_d, int64_t cap, const int32_t* slot_of_split,
                             int32_t* splits, int32_t sstride, int32_t rbshift) {
  const int64_t nsplit = *nsplit_d < cap ? *nsplit_d : cap;
  const int lane = lane_id();
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t sidx = w0; sidx < nsplit; sidx += nw) {
    const int32_t k = slot_of_split[sidx];
    const int64_t a0 = slot_begin(A, k);
    const int32_t al = (int32_t)(slot_begin(A, k + 1) - a0);
    const int32_t* col = A.ir + a0;
    int32_t* out = splits + sidx * sstride;
    for (int32_t e = lane; e < al; e += kWave) {
      const int32_t cur = col[e] >> rbshift;
      const int32_t prev = e == 0 ? -1 : (col[e - 1] >> rbshift);
      for (int32_t b = prev + 1; b <= cur; ++b) out[b] = e;
    }
    const int32_t last = al > 0 ? (col[al - 1] >> rbshift) : -1;
    for (int32_t b = last + 1 + lane; b < sstride; b += kWave) out[b] = al;
  }
}

// mults[t] = number of multiplications of output column (slot) t.  Groups
// of 8 lanes take one slot each (most columns hold a few B entries); slots
// with more than kLongSlot entries are listed for whole waves instead
// (k_slot_mults_long), so a long column holds up no group.  The total goes
// to *total with one atomic per workgroup.
constexpr int64_t kLongSlot = 512;

__device__ __forceinline__ void add_total(int64_t acc, bool mine, unsigned long long* total) {
  __shared__ unsigned long long s_acc;
  if (threadIdx.x == 0) s_acc = 0;
  __syncthreads();
  if (mine && acc) atomicAdd(&s_acc, (unsigned long long)acc);
  __syncthreads();
  if (threadIdx.x == 0 && s_acc) atomicAdd(total, s_acc);
}

__global__ void k_slot_mults(Operand B, const int32_t* bq_alen, int64_t nslots, int64_t* mults,
                             unsigned long long* total, int32_t* longs, unsigned long long* nlong) {
  constexpr int G = 8;
  const int gl = lane_id() & (G - 1);
  const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = (int64_t)gridDim.x * blockDim.x / G;
  int64_t acc = 0;
  for (int64_t t = grp; t < nslots; t += ngrp) {
    const int64_t b0 = slot_begin(B, t), b1 = slot_begin(B, t + 1);
    if (b1 - b0 > kLongSlot) {
      if (gl == 0) longs[atomicAdd(nlong, 1ull)] = (int32_t)t;
      continue;
    }
    int64_t s = 0;
    for (int64_t q = b0 + gl; q < b1; q += G) s += bq_alen[q];
#pragma unroll
    for (int d = 1; d < G; d <<= 1) s += __shfl_xor(s, d, G);
    if (gl == 0) {
      mults[t] = s;
      acc += s;
    }
  }
  add_total(acc, gl == 0, total);
}

__global__ void k_slot_mults_long(Operand B, const int32_t* bq_alen, const int32_t* longs,
                                  const unsigned long long* nlong, int64_t* mults, unsigned long long* total) {
  const int lane = lane_id();
  const int64_t n = (int64_t)*nlong;
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  int64_t acc = 0;
  for (int64_t i = wave; i < n; i += nwaves) {
    const int32_t t = longs[i];
    const int64_t b0 = slot_begin(B, t), b1 = slot_begin(B, t + 1);
    int64_t s = 0;
    for (int64_t q = b0 + lane; q < b1; q += kWave) s += bq_alen[q];
    s = wave_sum(s);
    if (lane == 0) {
      mults[t] = s;
      acc += s;
    }
  }
  add_total(acc, lane == 0, total);
}

// Counting sort of slots into bins: histogram, offsets, fill.
__global__ void k_bin_count(const int64_t* mults, int64_t nslots, BinCfg cfg, unsigned long long* counts) {
  __shared__ unsigned hist[kNumBins];
  for (int i = threadIdx.x; i < kNumBins; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nslots; t += stride)
    atomicAdd(&hist[bin_of(mults[t], cfg)], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kNumBins; i += blockDim.x)
    if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
}

// Each thread ranks kFillPer slots per round in LDS, so a workgroup reserves
// its ranges of the bins once per blockDim * kFillPer slots.  Every
// workgroup derives the bin offsets from the counts itself; the first one
// also stores them (binoff, kNumBins + 1 entries).  fill must be zero.
constexpr int kFillPer = 8;
__global__ void k_bin_fill(const int64_t* mults, int64_t nslots, BinCfg cfg, const unsigned long long* counts,
                           int64_t* binoff, unsigned long long* fill, int32_t* list) {
  __shared__ unsigned hist[kNumBins];
  __shared__ int64_t base[kNumBins];
  __shared__ int64_t off[kNumBins + 1];
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < kNumBins; ++i) {
      off[i] = run;
      run += (int64_t)counts[i];
    }
    off[kNumBins] = run;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i <= kNumBins; i += blockDim.x) binoff[i] = off[i];
  const int64_t span = (int64_t)blockDim.x * kFillPer;
  for (int64_t t0 = (int64_t)blockIdx.x * span; t0 < nslots; t0 += (int64_t)gridDim.x * span) {
    for (int i = threadIdx.x; i < kNumBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    int b[kFillPer];
    unsigned rank[kFillPer];
#pragma unroll
    for (int k = 0; k < kFillPer; ++k) {
      const int64_t t = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      b[k] = t < nslots ? bin_of(mults[t], cfg) : -1;
      rank[k] = b[k] >= 0 ? atomicAdd(&hist[b[k]], 1u) : 0u;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumBins; i += blockDim.x)
      if (hist[i]) base[i] = off[i] + (int64_t)atomicAdd(&fill[i], (unsigned long long)hist[i]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kFillPer; ++k)
      if (b[k] >= 0) list[base[b[k]] + rank[k]] = (int32_t)(t0 + (int64_t)k * blockDim.x + threadIdx.x);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ product iteration
// Work on one output column is spread over groups of G lanes (G a power of
// two, at most 64); each group takes one stored B(k,j) at a time and its G
// lanes stride through A(:,k).  Only rows in [r0, r1) are visited (a part
// of the row space); the start inside A(:,k) is found by binary search.
__device__ __forceinline__ int pick_group(int64_t mults, int64_t nq, int blk) {
  int64_t avg = nq > 0 ? (mults + nq - 1) / nq : 1;
  int g = 1;
  while (g < avg && g < kWave && g < blk) g <<= 1;
  return g;
}

__device__ __forceinline__ int32_t lower_bound_i32(const int32_t* a, int32_t n, int32_t key) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Where the products of one output column come from.  For every stored
// B(k,j) (index q): the start and length of A(:,k), and for long columns of
// A a row of the split table, whose entry b is the first position in A(:,k)
// with row >= b * 2^rbshift (b = 0..nblk; the last entry is the length).
// Parts of the row space start and end on those block boundaries, so a
// part's range inside a long column costs two loads; short columns are
// filtered entry by entry.
struct ProdSrc {
  const int32_t* air;
  const int64_t* a0;
  const int32_t* alen;
  const int32_t* split;
  const int32_t* splits;
  int32_t sstride;
  int32_t rbshift;
  int32_t m;
  int32_t off32;  // 1: positions in A fit 29 bits, loads take 32-bit byte offsets
};

// A's row and value at position o through a 32-bit byte offset from the base
// (valid when o < 2^29, so o * 8 does not wrap).
__device__ __forceinline__ int32_t load_row32(const int32_t* air, uint32_t o) {
  return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(air) + (o << 2));
}
template <typename T>
__device__ __forceinline__ T load_val32(const T* an, uint32_t o) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(an) + o * (uint32_t)sizeof(T));
}


// Block-cooperative iteration over the products of one output column.
// The column's stored B entries are taken in chunks of kQChunk: all threads
// first load, in parallel, each entry's range in A (start, length -- from
// the split table for long columns of A -- and B's value) into an LDS range
// list with a prefix sum of the lengths; then the products of the chunk are
// numbered 0..total-1 and taken in windows of 64 (one per lane of a wave),
// U windows per wave and round.  A lane finds the range of its product by a
// binary search over a short stretch of the list (see below), then loads
// A's row and value.  The work of the U windows is laid out in phases
// (search bounds, searches, range data, loads, callback) so that the loads
// of one phase are in flight together: a round costs a few LDS latencies
// and one global-memory latency for up to blockDim*U products.
// qidx (if given) lists the B entries to visit: qidx[b0, b1) instead of
// b0 .. b1-1.
// f receives the U products of a lane at once: rows r[u] (-1: none, e.g.
// past the end or outside [r0, r1)), A's values a[u] and B's values b[u].
// Must be called by every thread of the workgroup (it contains barriers);
// chunks hold min(blockDim.x, QC) entries, QC the capacity of the range list
// (kQChunk, or kQChunkWide for columns with very many B entries per product).
constexpr int kQChunk = 256;
constexpr int kQChunkWide = 512;

constexpr int kWinTab = 512;  // windows of 64 products with a table entry
constexpr int64_t kFilter = 1ll << 62;  // range start flag: filter rows one by one

template <int QC>
struct RangeLdsT {
  int64_t start[QC];  // position in A (| kFilter for unsplit columns)
  int32_t pref[QC + 1];
  double bval[QC];  // B's value, stored in the first bytes of each slot
  int16_t wst[kWinTab];  // range holding product 64 k
};
using RangeLds = RangeLdsT<kQChunk>;
// LDS that the wide range list takes beyond the ordinary one.
constexpr int64_t kWideExtraLds = sizeof(RangeLdsT<kQChunkWide>) - sizeof(RangeLdsT<kQChunk>);

// Adapts a per-product callback f(r, a, b) to the batch form.
template <int U, class F>
struct EachProduct {
  F f;
  template <typename T>
  __device__ __forceinline__ void operator()(const int32_t (&r)[U], const T (&a)[U], const T (&b)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (r[u] >= 0) f(r[u], a[u], b[u]);
  }
};
template <int U, class F>
__device__ __forceinline__ EachProduct<U, F> each_product(F f) {
  return EachProduct<U, F>{f};
}

// Range search of a window.  At set-up every range writes its index into
// the window table for each window (64 products) whose first product it
// holds (the first kWinTab windows).
//  WAVE_RUNS: each wave takes U consecutive windows per round.  The range
//    of the wave's first product (s0) comes from the table (else a binary
//    search); the lanes load the next 64 range starts, and ballots give each
//    window the ranges that start inside it, so a window inside one range
//    needs no search.  A round inside one range skips all of this and loads
//    consecutive entries.  (If all 64 loaded starts are inside the round,
//    the search runs over all ranges after s0.)
//  otherwise: windows are dealt round robin to the waves, and the table
//    bounds each window's search by the ranges of its first product and of
//    the next window's first product.
// With REUSE the range list left in R by the previous call for the same
// column and row range is used as is (the column must fit one chunk).
// Row-only passes (LOADA false) load through 32-bit byte offsets when
// S.off32 is set; value passes do so only with VAL32 (a separate kernel
// instantiation, so that the 64-bit path's registers are not held too).
template <int U, typename T, bool LOADA, bool LOADB, bool REUSE = false, bool WAVE_RUNS = false, bool VAL32 = false,
          int QC, class F>
__device__ __forceinline__ void block_products(const ProdSrc& S, const T* an, const T* bn, int64_t b0, int64_t b1,
                                               int32_t r0, int32_t r1, bool full, RangeLdsT<QC>& R, int64_t* red,
                                               const int32_t* qidx, F&& f) {
  const int qchunk = (int)blockDim.x < QC ? (int)blockDim.x : QC;
  const int lane = lane_id();
  const int32_t nwin = (int32_t)blockDim.x / kWave;
  const int32_t wid = __builtin_amdgcn_readfirstlane((int32_t)threadIdx.x / kWave);
  for (int64_t qc = b0; qc < b1; qc += qchunk) {
    const int nq = (int)(b1 - qc < qchunk ? b1 - qc : qchunk);
    int32_t mylen = 0;
    if (!REUSE && (int)threadIdx.x < nq) {
      const int i = threadIdx.x;
      const int64_t q = qidx ? (int64_t)qidx[qc + i] : qc + i;
      const int64_t a0 = S.a0[q];
      int32_t e0 = 0, e1 = S.alen[q];
      int64_t flt = 0;
      if (!full) {
        const int32_t sid = S.splits ? S.split[q] : -1;
        if (sid >= 0) {
          const int32_t* sp = S.splits + (int64_t)sid * S.sstride;
          e0 = sp[r0 >> S.rbshift];
          e1 = sp[r1 >= S.m ? S.sstride - 1 : (r1 >> S.rbshift)];
        } else {
          flt = kFilter;
        }
      }
      R.start[i] = (a0 + e0) | flt;
      if constexpr (LOADB) reinterpret_cast<T*>(&R.bval[i])[0] = bn[q];
      mylen = e1 - e0;
    }
    if (!REUSE) {
      int64_t total64;
      const int64_t ex = block_excl_scan1((int64_t)mylen, red, &total64);
      if ((int)threadIdx.x < nq) {
        R.pref[threadIdx.x] = (int32_t)ex;
        // windows whose first product falls in this range
        const int64_t k1 = (ex + mylen + kWave - 1) / kWave;
        for (int64_t k = (ex + kWave - 1) / kWave; k < k1 && k < kWinTab; ++k) R.wst[k] = (int16_t)threadIdx.x;
      }
      if (threadIdx.x == 0) R.pref[nq] = (int32_t)total64;
      __syncthreads();
    }
    const int32_t total = R.pref[nq];
    for (int32_t base = 0; base < total; base += (int32_t)blockDim.x * U) {
      const int32_t pw = base + wid * (U * kWave);
      // phase 1: search bounds [lo, lo + n) of every window (wave-uniform)
      int lo[U], n[U];
      if constexpr (WAVE_RUNS) {
        int s0 = 0, s1 = 1;
        if (pw < total) {
          int l = 0;
          if (pw / kWave < kWinTab) {
            l = R.wst[pw / kWave];
          } else {
            int h = nq;
            while (h - l > 1) {
              const int mid = (l + h) >> 1;
              if (R.pref[mid] <= pw)
                l = mid;
              else
                h = mid;
            }
          }
          s0 = __builtin_amdgcn_readfirstlane(l);
          const int j = s0 + 1 + lane;
          const int32_t bj = j <= nq ? R.pref[j] : 0x7fffffff;
          const uint64_t in_round = __ballot(bj < pw + U * kWave);
          if (in_round == 0 && pw + U * kWave <= total) {
            // the whole round lies in range s0: consecutive products, no search
            const int64_t st = R.start[s0];
            const int64_t eb = (st & (kFilter - 1)) + (pw - R.pref[s0]) + lane;
            const bool fl1 = (st & kFilter) != 0;
            const T b1 = LOADB ? reinterpret_cast<const T*>(&R.bval[s0])[0] : T(0);
            int32_t r[U];
            T a[U], bv[U];
            if (VAL32 || (!LOADA && S.off32)) {  // VAL32: the caller's A fits 29-bit positions
              const uint32_t eb32 = (uint32_t)eb;
#pragma unroll
              for (int u = 0; u < U; ++u) {
                r[u] = load_row32(S.air, eb32 + (uint32_t)(u * kWave));
                a[u] = LOADA ? load_val32(an, eb32 + (uint32_t)(u * kWave)) : T(0);
                bv[u] = b1;
              }
            } else {
#pragma unroll
              for (int u = 0; u < U; ++u) {
                r[u] = S.air[eb + u * kWave];
                a[u] = LOADA ? an[eb + u * kWave] : T(0);
                bv[u] = b1;
              }
            }
            if (fl1) {
#pragma unroll
              for (int u = 0; u < U; ++u)
                if (r[u] < r0 || r[u] >= r1) r[u] = -1;
            }
            f(r, a, bv);
            continue;
          }
          if (in_round == ~0ull) {
            s1 = nq + 1;
          } else {
            // each window: the ranges starting inside it
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int32_t p0 = pw + u * kWave;
              lo[u] = s0 + __popcll(__ballot(bj <= p0));
              n[u] = s0 + __popcll(__ballot(bj < p0 + kWave)) + 1 - lo[u];
            }
            s1 = -1;
          }
        }
        if (s1 >= 0) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            lo[u] = s0;
            n[u] = s1 - s0;
          }
        }
      } else {
        // all table reads first (one LDS latency), then the bounds
        int tl[U], th[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t k = base / kWave + u * nwin + wid;
          const int32_t kc = k < kWinTab - 1 ? k : kWinTab - 2;
          tl[u] = R.wst[kc];
          th[u] = R.wst[kc + 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t p0 = base + (u * nwin + wid) * kWave;
          const int32_t k = p0 / kWave;
          int l = 0, h = 1;
          if (p0 >= total) {
          } else if (k + 1 < kWinTab && p0 + kWave < total) {
            l = tl[u];
            h = th[u] + 1;
          } else {
            l = k < kWinTab ? tl[u] : 0;
            h = nq;
          }
          lo[u] = __builtin_amdgcn_readfirstlane(l);
          n[u] = __builtin_amdgcn_readfirstlane(h) - lo[u];
        }
      }
      // phase 2: last range with start <= p (uniform trip counts)
      int32_t p[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t pp = (WAVE_RUNS ? pw + u * kWave : base + (u * nwin + wid) * kWave) + lane;
        p[u] = pp < total ? pp : total - 1;
        int pos = lo[u];
        for (int m = n[u]; m > 1;) {
          const int half = m >> 1;
          if (R.pref[pos + half] <= p[u]) pos += half;
          m -= half;
        }
        lo[u] = pos;
        if (pp >= total) p[u] = -1;
      }
      // phase 3: range data; phase 4: A's row and value
      int64_t st[U];
      int32_t d[U];
      int32_t r[U];
      T a[U], bv[U];
      bool fl[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        st[u] = R.start[lo[u]];
        const int32_t pf = R.pref[lo[u]];
        fl[u] = (st[u] & kFilter) != 0;
        d[u] = (p[u] < 0 ? total - 1 : p[u]) - pf;
        bv[u] = LOADB ? reinterpret_cast<const T*>(&R.bval[lo[u]])[0] : T(0);
      }
      if (VAL32 || (!LOADA && S.off32)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          r[u] = -1;
          a[u] = T(0);
          // windows wholly past the end load nothing (wave-uniform test)
          if ((WAVE_RUNS ? pw + u * kWave : base + (u * nwin + wid) * kWave) < total) {
            const uint32_t o = (uint32_t)st[u] + (uint32_t)d[u];  // the flag is above bit 31
            r[u] = load_row32(S.air, o);
            if constexpr (LOADA) a[u] = load_val32(an, o);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          r[u] = -1;
          a[u] = T(0);
          if ((WAVE_RUNS ? pw + u * kWave : base + (u * nwin + wid) * kWave) < total) {
            const int64_t e = (st[u] & (kFilter - 1)) + d[u];
            r[u] = S.air[e];
            if constexpr (LOADA) a[u] = an[e];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (p[u] < 0 || (fl[u] && (r[u] < r0 || r[u] >= r1))) r[u] = -1;
      f(r, a, bv);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t hash_row(int32_t r, int log2s) {
  return ((uint32_t)r * 0x9E3779B1u) >> (32 - log2s);
}

// ------------------------------------------------------------------ count: tiny (one wave)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Group-wide helpers over G lanes: the whole wave (G = 64) or one of its
// aligned halves (G = 32); exchanges stay inside the group.
// Inclusive scan with op by DPP: shifts by 1, 2, 4, 8 inside each 16-lane
// row, then the last lane of row 0 (2) is added into row 1 (3), and for
// G = 64 lane 31 into rows 2 and 3.  Lanes without a source receive ident.
template <int G, class Op>
__device__ __forceinline__ int group_scan(int v, int ident, Op op) {
  static_assert(G == 32 || G == 64, "groups of 32 or 64 lanes");
  v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x111, 0xF, 0xF, false));  // row_shr:1
  v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x112, 0xF, 0xF, false));  // row_shr:2
  v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x114, 0xF, 0xF, false));  // row_shr:4
  v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x118, 0xF, 0xF, false));  // row_shr:8
  v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  if constexpr (G == 64) v = op(v, __builtin_amdgcn_update_dpp(ident, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return v;
}

// Value of the next lane (lane + 1; 0 in lane 63) by a DPP wave shift.
template <typename T>
__device__ __forceinline__ T lane_next(T v) {
  if constexpr (sizeof(T) == 4) {
    const int u = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, u, 0x130, 0xF, 0xF, false));  // wave_shl:1
  } else {
    static_assert(sizeof(T) == 8, "32- or 64-bit values");
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x130, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x130, 0xF, 0xF, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

template <int G>
__device__ __forceinline__ int group_incl_scan(int v, int) {
  return group_scan<G>(v, 0, [](int x, int y) { return x + y; });
}

template <int G, typename K>
__device__ __forceinline__ K group_sort(K key, int gl) {  // ascending bitonic sort, one key per lane
#pragma unroll
  for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const K other = xor_lane(key, j);
      const bool up = (gl & k) == 0;
      const bool lower = (gl & j) == 0;
      const K mn = other < key ? other : key;
      const K mx = other < key ? key : other;
      key = (lower == up) ? mn : mx;
    }
  }
  return key;
}

// One tiny column (at most G products) in a group of G lanes: the group
// gathers every product into LDS; the count (COUNT) inserts the rows into a
// small LDS table and counts the distinct ones; the numeric pass sorts the
// (row, product index) keys, sums each run of equal rows in product order
// -- the order of Algorithm 1 -- and writes the column.  The column's B
// range [b0, b1) and output offset come from the caller.
template <int G, int SR, typename T, bool COUNT>
__device__ __forceinline__ void tiny_column(const Operand& A, const Operand& B, const int64_t* bq_a0,
                                            const int32_t* bq_alen, int32_t t, int64_t b0, int64_t b1,
                                            int64_t obase, int64_t* cnt, int32_t* cir, T* cnum, int32_t* s_row,
                                            int32_t* s_aux, T* s_val, uint32_t* s_tab) {
  using S = Semiring<SR, T>;
  constexpr bool kVal = SR != SPX_OR_AND;
  const int lane = lane_id();
  const int gl = lane & (G - 1);
  const int gb = lane & ~(G - 1);
  s_row += gb;
  s_aux += gb;
  s_val += gb;
  const T* an = (const T*)A.num;
  const T* bn = (const T*)B.num;
  int total = 0;
  for (int64_t qc = b0; qc < b1; qc += G) {
    const int64_t q = qc + gl;
    const bool inq = q < b1;
    // each lane loads its own B entry's A range (and value) next to its
    // length; the lanes that take the products get them by shuffles
    const int al = inq ? bq_alen[q] : 0;
    const int64_t qa0 = inq ? bq_a0[q] : 0;
    T qb = T(0);
    if constexpr (kVal && S::kUsesB) qb = inq ? bn[q] : T(0);
    const int incl = group_incl_scan<G>(al, gl);
    const int excl = incl - al;
    // the group's total: its last lane, read as a scalar (lanes of an idle
    // half may hold stale values, which only that half would read)
    const int ctot = G == 64 ? __builtin_amdgcn_readlane(incl, 63)
                             : (lane < 32 ? __builtin_amdgcn_readlane(incl, 31) : __builtin_amdgcn_readlane(incl, 63));
    if (ctot == 0) continue;
    s_aux[gl] = -1;
    wave_sync();
    if (al > 0 && excl < G) s_aux[excl] = gl;
    wave_sync();
    const int o = group_scan<G>(s_aux[gl], -1, [](int x, int y) { return x > y ? x : y; });
    const int src = o < 0 ? 0 : o;
    const int ostart = __shfl(excl, src, G);
    const int64_t ea0 = __shfl(qa0, src, G);
    T bv = T(0);
    if constexpr (kVal && S::kUsesB) bv = __shfl(qb, src, G);
    if (gl < ctot && total + gl < G) {
      const int64_t e = ea0 + (gl - ostart);
      s_row[total + gl] = A.ir[e];
      if constexpr (kVal) {
        const T a = S::kUsesA ? an[e] : T(0);
        s_val[total + gl] = S::mul(a, bv);
      }
    }
    total += ctot;
    wave_sync();
  }
  if (total > G) total = G;  // cannot happen: the caller checked the column's products
  if constexpr (COUNT) {
    // distinct rows: each lane inserts its product's row into the group's
    // table of 2G slots (linear probing; a row is below 2^31, so the empty
    // mark never matches); the lanes that claimed a slot hold the distinct rows
    uint32_t* tab = s_tab + 2 * gb;
    tab[gl] = 0xffffffffu;
    tab[gl + G] = 0xffffffffu;
    wave_sync();
    bool fresh = false;
    if (gl < total) {
      const uint32_t r = (uint32_t)s_row[gl];
      uint32_t h = (r * 0x9E3779B1u) >> (32 - (G == 64 ? 7 : 6));
      for (;;) {
        const uint32_t old = atomicCAS(&tab[h], 0xffffffffu, r);
        if (old == 0xffffffffu) {
          fresh = true;
          break;
        }
        if (old == r) break;
        h = (h + 1) & (2 * G - 1);
      }
    }
    const uint64_t gmask = G == 64 ? ~0ull : (0xffffffffull << gb);
    const uint64_t fm = __ballot(fresh) & gmask;
    if (gl == 0) cnt[t] = __popcll(fm);
    wave_sync();
    return;
  }
  // sort (row, product index): 32-bit keys when the rows leave 6 bits for
  // the index (the count needs the rows only)
  int32_t row;
  int idx;
  if (COUNT || A.m <= (1ll << 25)) {
    const uint32_t k32 = gl < total ? (COUNT ? (uint32_t)s_row[gl] : ((uint32_t)s_row[gl] << 6) | gl) : 0xffffffffu;
    const uint32_t key = group_sort<G, uint32_t>(k32, gl);
    row = COUNT ? (int32_t)key : (int32_t)(key >> 6);
    idx = COUNT ? 0 : (int)(key & 63u);
  } else {
    const uint64_t k64 = gl < total ? (((uint64_t)(uint32_t)s_row[gl]) << 32) | (uint32_t)gl : ~0ull;
    const uint64_t key = group_sort<G, uint64_t>(k64, gl);
    row = (int32_t)(key >> 32);
    idx = (int)(key & 0xffffffffu);
  }
  // the previous lane's row (DPP wave shift; lane 0 of a group never uses it)
  const int32_t prev = __builtin_amdgcn_update_dpp(0, row, 0x138, 0xF, 0xF, false);  // wave_shr:1
  const bool valid = gl < total;
  const bool head = valid && (gl == 0 || prev != row);
  const uint64_t gmask = G == 64 ? ~0ull : (0xffffffffull << gb);
  const uint64_t hm = __ballot(head) & gmask;
  if (COUNT) {
    if (gl == 0) cnt[t] = __popcll(hm);
  } else {
    // every lane holds its sorted product's value; a head lane folds its run
    // left to right (product order) from the values of the lanes after it
    const uint64_t hg = hm >> gb;  // the group's heads, bit gl for lane gl
    const uint64_t later = gl + 1 < 64 ? hg >> (gl + 1) : 0ull;
    const int run = !head ? 0 : (later ? __ffsll((long long)later) : total - gl);
    T acc = T(0);
    if constexpr (kVal) {
      const T v = valid ? s_val[idx] : T(0);
      acc = v;
      int mr = run;  // longest run of the wave
#pragma unroll
      for (int j = 32; j > 0; j >>= 1) {
        const int t = (int)xor_lane_u32((uint32_t)mr, j);
        mr = t > mr ? t : mr;
      }
      const int maxrun = __builtin_amdgcn_readfirstlane(mr);
      T x = v;  // after d steps: the value of lane gl + d (inside the group while d < run)
      for (int d = 1; d < maxrun; ++d) {
        x = lane_next(x);
        if (d < run) acc = S::add(acc, x);
      }
    }
    if (head) {
      const int64_t o = obase + __popcll(hm & lanemask_lt());
      cir[o] = row;
      if constexpr (kVal) cnum[o] = acc;
    }
  }
  wave_sync();
}

// Tiny columns (at most 64 products), by pairs of consecutive columns of
// the bin: two columns of at most 32 products each share a wave (one per
// half), otherwise they are done one after the other.  A wave takes up to
// 64 pairs at a time (fewer when the bin is too small to give every wave
// 64): lane k loads pair k's column ids, products, B ranges and output
// offsets into the wave's LDS table (two load levels for all of them), and
// the pair loop reads them from there, so a column waits only on its B
// entries' A ranges and then A's rows and values.
template <int SR, typename T, bool COUNT>
__global__ void __launch_bounds__(256) k_tiny(Operand A, Operand B, const int64_t* bq_a0, const int32_t* bq_alen,
                                              const int64_t* mults, const int32_t* list, const int64_t* binoff,
                                              int64_t* cnt, const int64_t* off, int32_t* cir, T* cnum) {
  __shared__ int32_t s_row[4][kWave];
  __shared__ int32_t s_aux[4][kWave];
  __shared__ T s_val[4][kWave];
  struct PairRow {
    int32_t t[2];
    int32_t m[2];  // products (a tiny column's fit 32 bits)
    int64_t b0[2], b1[2], o[2];
  };
  __shared__ PairRow s_pair[4][kWave];
  __shared__ uint32_t s_tab[4][2 * kWave];  // the count's distinct-row tables
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t beg = binoff[kBinTiny], end = binoff[kBinTiny + 1];
  const int64_t npairs = (end - beg + 1) / 2;
  const int64_t wave = (int64_t)blockIdx.x * 4 + w, nwaves = (int64_t)gridDim.x * 4;
  const int64_t per = std::min<int64_t>(kWave, std::max<int64_t>(1, (npairs + nwaves - 1) / nwaves));
  for (int64_t c0 = wave * per; c0 < npairs; c0 += nwaves * per) {
    {  // lane k: pair c0 + k
      const int64_t pos = beg + 2 * (c0 + lane);
      PairRow r{};
      r.m[1] = -1;  // no second column
      if (lane < per && c0 + lane < npairs) {
        for (int h = 0; h < 2; ++h) {
          if (pos + h >= end) break;
          const int32_t t = list[pos + h];
          r.t[h] = t;
          r.m[h] = (int32_t)mults[t];
          r.b0[h] = slot_begin(B, t);
          r.b1[h] = slot_begin(B, t + 1);
          r.o[h] = COUNT ? 0 : off[t];
        }
      }
      s_pair[w][lane] = r;
    }
    wave_sync();
    const int np = (int)std::min<int64_t>(per, npairs - c0);
    for (int k = 0; k < np; ++k) {
      const PairRow& r = s_pair[w][k];
      const int32_t m1 = __builtin_amdgcn_readfirstlane(r.m[1]);
      const bool has1 = m1 >= 0;
      const int32_t m0 = __builtin_amdgcn_readfirstlane(r.m[0]);
      if (has1 && m0 <= 32 && m1 <= 32) {
        const int h = lane < 32 ? 0 : 1;
        tiny_column<32, SR, T, COUNT>(A, B, bq_a0, bq_alen, r.t[h], r.b0[h], r.b1[h], r.o[h], cnt, cir, cnum,
                                      s_row[w], s_aux[w], s_val[w], s_tab[w]);
      } else {
        tiny_column<64, SR, T, COUNT>(A, B, bq_a0, bq_alen, r.t[0], r.b0[0], r.b1[0], r.o[0], cnt, cir, cnum,
                                      s_row[w], s_aux[w], s_val[w], s_tab[w]);
        if (has1)
          tiny_column<64, SR, T, COUNT>(A, B, bq_a0, bq_alen, r.t[1], r.b0[1], r.b1[1], r.o[1], cnt, cir, cnum,
                                        s_row[w], s_aux[w], s_val[w], s_tab[w]);
      }
    }
    wave_sync();  // the table is rewritten for the next 64 pairs
  }
}

// ------------------------------------------------------------------ count: hash
// One workgroup per column; key-only open-addressing table of 2^log2s
// slots (at least twice the number of products).  Columns listed before
// position `multi_end` also get their distinct rows counted per row block.
__global__ void k_count_hash(Operand B, ProdSrc S, const int64_t* mults,
                             const int32_t* list, const int64_t* binoff, int bin, int log2s, int64_t multi_end,
                             int rbshift, int64_t nblk, uint32_t* blkcnt, int64_t* cnt, unsigned* err) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint32_t* keys = (uint32_t*)lds;
  const uint32_t TS = 1u << log2s;
  uint32_t* lblk = keys + TS;  // per-block counters when they fit
  __shared__ int64_t red[1024 / kWave + 1];
  __shared__ RangeLds s_rng;
  const int64_t beg = binoff[bin], end = binoff[bin + 1];
  for (int64_t pos = beg + blockIdx.x; pos < end; pos += gridDim.x) {
    const int32_t t = list[pos];
    const int64_t b0 = slot_begin(B, t), b1 = slot_begin(B, t + 1);
    const bool want_blk = pos < multi_end;
    const bool lds_blk = nblk <= 1024;
    for (uint32_t i = threadIdx.x; i < TS; i += blockDim.x) keys[i] = 0xffffffffu;
    if (want_blk && lds_blk)
      for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) lblk[i] = 0;
    __syncthreads();
    int64_t mine = 0;
    block_products<4, int, false, false, false, true>(S, nullptr, nullptr, b0, b1, 0, 0, true, s_rng, red, nullptr,
                                                      each_product<4>([&](int32_t r, int, int) {
      if (r < 0) return;
      uint32_t h = hash_row(r, log2s);
      for (uint32_t probe = 0; probe < TS; ++probe) {
        const uint32_t old = atomicCAS(&keys[h], 0xffffffffu, (uint32_t)r);
        if (old == 0xffffffffu) {
          ++mine;
          return;
        }
        if (old == (uint32_t)r) return;
        h = (h + 1) & (TS - 1);
      }
      atomicOr(err, 2u);
    }));
    __syncthreads();
    int64_t total;
    block_excl_scan1(mine, red, &total);
    if (threadIdx.x == 0) cnt[t] = total;
    if (want_blk) {
      uint32_t* dst = blkcnt + (pos - binoff[0]) * nblk;
      for (uint32_t i = threadIdx.x; i < TS; i += blockDim.x) {
        const uint32_t key = keys[i];
        if (key != 0xffffffffu) {
          if (lds_blk)
            atomicAdd(&lblk[key >> rbshift], 1u);
          else
            atomicAdd(&dst[key >> rbshift], 1u);
        }
      }
      if (lds_blk) {
        __syncthreads();
        for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) dst[i] = lblk[i];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ count: bitmap
// One workgroup per heavy column; an LDS bitmap over (a chunk of) the row
// space marks every row that receives a product.  Popcounts give the exact
// column count and the per-row-block counts used to cut parts.
__global__ void k_count_bitmap(Operand B, ProdSrc S, const int64_t* mults, const int32_t* list, const int64_t* binoff,
                               int64_t m, int chunk_log2, int rbshift, int64_t nblk, uint32_t* blkcnt,
                               unsigned long long* cnt, uint32_t* gbm, int64_t gwords, unsigned long long* qctr) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint32_t* bm = (uint32_t*)lds;
  const int64_t chunk_rows = 1ll << chunk_log2;  // a multiple of the row block
  const int64_t nchunks = (m + chunk_rows - 1) >> chunk_log2;
  const int blk_per_chunk = (int)(chunk_rows >> rbshift);
  uint32_t* lblk = bm + (chunk_rows >> 5);
  __shared__ int64_t red[1024 / kWave + 1];
  __shared__ RangeLds s_rng;
  const int64_t beg = binoff[0], end = binoff[kBinHash0];
  const int64_t ncols = end - beg;
  // workgroup w works on row chunk w mod nchunks (the grid is a multiple of
  // nchunks): workgroups are placed on the XCDs round robin, so each XCD's L2
  // serves one slice of A's rows.  The chunk's columns are handed out one at
  // a time by its counter qctr[chunk] (zero at launch), in list order, which
  // puts the heaviest columns first.
  const int64_t chunk = blockIdx.x % nchunks;
  __shared__ int64_t s_ci;
  for (;;) {
    if (threadIdx.x == 0) s_ci = (int64_t)atomicAdd(&qctr[chunk], 1ull);
    __syncthreads();
    const int64_t ci = s_ci;
    if (ci >= ncols) break;
    const int64_t pos = beg + ci;
    const int64_t c0 = chunk * chunk_rows;
    const int64_t c1 = c0 + chunk_rows < m ? c0 + chunk_rows : m;
    const int32_t t = list[pos];
    const int64_t b0 = slot_begin(B, t), b1 = slot_begin(B, t + 1);
    uint32_t* dst = blkcnt + (pos - beg) * nblk;
    const int words = (int)((c1 - c0 + 31) >> 5);
    {  // 16-byte LDS stores (the LDS base is 16-byte aligned), then the ragged end
      const int w4 = words >> 2;
      for (int i = threadIdx.x; i < w4; i += blockDim.x) reinterpret_cast<uint4*>(bm)[i] = make_uint4(0u, 0u, 0u, 0u);
      for (int i = (w4 << 2) + (int)threadIdx.x; i < words; i += blockDim.x) bm[i] = 0;
    }
    for (int i = threadIdx.x; i < blk_per_chunk; i += blockDim.x) lblk[i] = 0;
    __syncthreads();
    block_products<4, int, false, false, false, true>(S, nullptr, nullptr, b0, b1, (int32_t)c0, (int32_t)c1, nchunks == 1, s_rng,
                                         red, nullptr, each_product<4>([&](int32_t r, int, int) {
      const uint32_t d = (uint32_t)(r - (int32_t)c0);
      if (d < (uint32_t)(c1 - c0)) atomicOr(&bm[d >> 5], 1u << (d & 31));
    }));
    __syncthreads();
    int64_t mine = 0;
    if (rbshift >= 11) {
      // a wave's 64 words (2048 rows, 64-aligned) lie in one row block:
      // one LDS add per wave instead of one per nonzero word at one address
      const int lane = lane_id();
      for (int w = (int)threadIdx.x - lane; w < words; w += blockDim.x) {
        const int i = w + lane;
        const int pc = i < words ? __popc(bm[i]) : 0;
        mine += pc;
        const int s = __builtin_amdgcn_readlane(wave_incl_scan(pc), 63);
        if (lane == 0 && s) atomicAdd(&lblk[((int64_t)w * 32) >> rbshift], (uint32_t)s);
      }
    } else {
      for (int i = threadIdx.x; i < words; i += blockDim.x) {
        const int pc = __popc(bm[i]);
        if (pc) {
          mine += pc;
          atomicAdd(&lblk[((int64_t)i * 32) >> rbshift], (uint32_t)pc);
        }
      }
    }
    int64_t ctot;
    block_excl_scan1(mine, red, &ctot);
    const int64_t bfirst = c0 >> rbshift;
    for (int i = threadIdx.x; i < blk_per_chunk; i += blockDim.x)
      if (bfirst + i < nblk) dst[bfirst + i] = lblk[i];
    if (threadIdx.x == 0 && ctot) atomicAdd(&cnt[t], (unsigned long long)ctot);
    if (gbm) {  // keep the column's row set for the numeric phase
      // whole 64-bit words (gwords is even and c0 a multiple of 64 rows, so g
      // is 8-byte aligned); a ragged chunk's last word is padded with zeros
      uint2* g = reinterpret_cast<uint2*>(gbm + ci * gwords + (c0 >> 5));
      const int w2 = (words + 1) >> 1;
      for (int i = threadIdx.x; i < w2; i += blockDim.x) {
        const int k = 2 * i;
        // streaming (non-temporal) stores: the bitmaps are read back only by the
        // numeric phase, so they need not displace A's gathered entries from L2
        const uint64_t pair = ((uint64_t)(k + 1 < words ? bm[k + 1] : 0u) << 32) | bm[k];
        __builtin_nontemporal_store(pair, reinterpret_cast<uint64_t*>(g) + i);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ parts
struct Part {
  int64_t off;   // first output position of the part in C
  int32_t t;     // slot of B / output column
  int32_t c;     // outputs in the part
  int32_t r0, r1;  // row range [r0, r1)
  int32_t mode;  // bit 0: 0 = bitmap, 1 = hash; bit 1: [b0, b0 + nb) indexes the bucket list
  int32_t slice; // row slice of the part (work queue), nslice = any
  int32_t bmi;   // index of the column's stored row bitmap, -1 if none
  int32_t nb;    // B entries of the column: [b0, b0 + nb) (or the part's bucket)
  int64_t b0;
};

struct PartCfg {
  int64_t L;       // LDS bytes per part
  int64_t m;
  int32_t sz;      // value bytes (0: pattern only)
  int32_t rbshift;
  int64_t nblk;
  int64_t slice_blocks;  // row blocks per slice (parts never straddle slices); 0: one slice
  int32_t nslice;
  int32_t pad;
};

__device__ __forceinline__ int64_t bitmap_bytes(const PartCfg& p, int64_t span, int64_t c) {
  const int64_t w = (span + 63) >> 6;
  return w * 8 + ((w * 2 + 7) & ~7ll) + c * (p.sz > 4 ? p.sz : 4) + 64;
}
__device__ __forceinline__ bool bitmap_ok(const PartCfg& p, int64_t span, int64_t c) {
  return c < 65536 && bitmap_bytes(p, span, c) <= p.L;
}
// Rows a hash-mode part may span for the two-level rank (longer: sorted).
constexpr int64_t kRankSpan = 1ll << 20;

__device__ __forceinline__ int64_t hash_bytes(const PartCfg& p, int64_t c) {
  int64_t p2 = 64;
  while (p2 < c) p2 <<= 1;
  const int64_t S = 2 * p2;
  return S * 4 + ((S * p.sz + 7) & ~7ll) + p2 * 10 + (kRankSpan >> 9) + (kRankSpan >> 11) + 64;
}
__device__ __forceinline__ bool hash_ok(const PartCfg& p, int64_t c) { return hash_bytes(p, c) <= p.L; }

__device__ __forceinline__ int choose_mode(const PartCfg& p, int64_t span, int64_t c) {
  const bool bok = bitmap_ok(p, span, c), hok = hash_ok(p, c);
  if (bok && hok) {
    const int64_t lg = c > 1 ? ceil_log2_u64((uint64_t)c) : 1;
    const int64_t bitmap_cost = ((span + 63) >> 6) * 3;
    const int64_t hash_cost = c * lg * (lg + 1) / 2;
    return bitmap_cost <= hash_cost ? 0 : 1;
  }
  return bok ? 0 : 1;
}

// Walks the row blocks of one multi-part column greedily: a part grows while
// it still fits the LDS budget in one of the two modes.  With emit == false
// only counts parts.
__device__ int64_t cut_parts(const PartCfg& p, const uint32_t* blk, int32_t t, int64_t base_off, bool emit, Part* out,
                             int32_t bmi, int64_t b0, int32_t nb, unsigned* err) {
  const int64_t RB = 1ll << p.rbshift;
  int64_t np = 0, run = 0;
  int64_t b = 0;
  while (b < p.nblk) {
    int64_t c = blk[b];
    int64_t e = b + 1;
    while (e < p.nblk) {
      if (p.slice_blocks && e % p.slice_blocks == 0) break;
      const int64_t c2 = c + blk[e];
      const int64_t r1 = (e + 1) * RB < p.m ? (e + 1) * RB : p.m;
      const int64_t span2 = r1 - b * RB;
      if (bitmap_ok(p, span2, c2) || hash_ok(p, c2)) {
        c = c2;
        ++e;
      } else {
        break;
      }
    }
    if (c > 0) {
      const int64_t r0 = b * RB;
      const int64_t r1 = e * RB < p.m ? e * RB : p.m;
      if (!bitmap_ok(p, r1 - r0, c) && !hash_ok(p, c)) atomicOr(err, 4u);
      if (emit) {
        Part P;
        P.off = base_off + run;
        P.t = t;
        P.c = (int32_t)c;
        P.r0 = (int32_t)r0;
        P.r1 = (int32_t)r1;
        P.mode = choose_mode(p, r1 - r0, c);
        P.slice = p.slice_blocks ? (int32_t)(b / p.slice_blocks) : 0;
        P.bmi = bmi;
        P.b0 = b0;
        P.nb = nb;
        out[np] = P;
      }
      ++np;
      run += c;
    }
    b = e;
  }
  return np;
}

// Number of parts of every non-tiny, nonempty column (list positions
// [0, npos)), or the parts themselves (emit).
// In the counting pass, setup_acc (if given) receives the sums over the cut
// columns of (B entries x parts) and of their multiplications, which tell
// how many range set-ups the multi-part launch makes per product.
__global__ void k_parts(Operand B, PartCfg p, PartCfg ps, const int32_t* list, int64_t npos, int64_t multi_begin, int64_t multi_end,
                        int64_t nbm, const int64_t* cnt, const int64_t* off, const uint32_t* blkcnt,
                        int64_t* nparts, const int64_t* poff, Part* parts, const int64_t* mults,
                        unsigned long long* setup_acc, unsigned* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool emit = parts != nullptr;
  unsigned long long my_setup = 0, my_mults = 0;
  for (int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pos < npos; pos += stride) {
    const int32_t t = list[pos];
    const int64_t c = cnt[t];
    int64_t np;
    if (c == 0) {
      np = 0;
    } else if (pos >= multi_begin && pos < multi_end && !(bitmap_ok(p, p.m, c) || hash_ok(p, c))) {
      const int64_t cb0 = slot_begin(B, t);
      np = cut_parts(p, blkcnt + (pos - multi_begin) * p.nblk, t, off[t], emit, emit ? parts + poff[pos] : nullptr,
                     pos - multi_begin < nbm ? (int32_t)(pos - multi_begin) : -1, cb0,
                     (int32_t)(slot_begin(B, t + 1) - cb0), err);
      if (setup_acc && np > 1) {
        my_setup += (unsigned long long)(slot_begin(B, t + 1) - cb0) * (unsigned long long)np;
        my_mults += (unsigned long long)mults[t];
      }
    } else {
      np = 1;
      const PartCfg& q = pos < multi_end ? p : ps;
      if (!emit && !(bitmap_ok(q, q.m, c) || hash_ok(q, c))) atomicOr(err, 4u);
      if (emit) {
        Part P;
        P.off = off[t];
        P.t = t;
        P.c = (int32_t)c;
        P.r0 = 0;
        P.r1 = (int32_t)q.m;
        P.mode = choose_mode(q, q.m, c);
        P.slice = q.nslice;  // full row range: any queue
        P.bmi = pos - multi_begin < nbm ? (int32_t)(pos - multi_begin) : -1;
        P.b0 = slot_begin(B, t);
        P.nb = (int32_t)(slot_begin(B, t + 1) - P.b0);
        parts[poff[pos]] = P;
      }
    }
    if (!emit) nparts[pos] = np;
  }
  if (setup_acc) {  // one pair of atomics per workgroup
    __shared__ unsigned long long s_acc[2];
    if (threadIdx.x < 2) s_acc[threadIdx.x] = 0;
    __syncthreads();
    if (my_setup) atomicAdd(&s_acc[0], my_setup);
    if (my_mults) atomicAdd(&s_acc[1], my_mults);
    __syncthreads();
    if (threadIdx.x < 2 && s_acc[threadIdx.x]) atomicAdd(&setup_acc[threadIdx.x], s_acc[threadIdx.x]);
  }
}

// ------------------------------------------------------------------ buckets
// With a tall-skinny B, every part of a cut column walks all of the column's
// B entries although the few rows of each A(:,k) reach few parts.  Bucket
// mode lists, per part, only the B entries whose A column has rows in the
// part's row range: about one list entry per multiplication instead of one
// range set-up per B entry and part.
//   k_bucket_map:   per cut column, the part of every row block (-1: none);
//   k_bucket<FILL>: per B entry of a cut column, each part it reaches gets a
//                   count (FILL false) or the entry's index (FILL true);
//   k_bucket_parts: points every part of a cut column at its bucket.
// Cut columns are the list positions [multi_begin, multi_end) with more
// than one part.
__global__ void k_bucket_map(PartCfg p, const int64_t* np, const int64_t* poff, int64_t multi_begin,
                             int64_t multi_end, const Part* parts, int32_t* map) {
  for (int64_t pos = multi_begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pos < multi_end;
       pos += (int64_t)gridDim.x * blockDim.x) {
    int32_t* mp = map + (pos - multi_begin) * p.nblk;
    for (int64_t b = 0; b < p.nblk; ++b) mp[b] = -1;
    if (np[pos] <= 1) continue;
    for (int64_t i = poff[pos]; i < poff[pos + 1]; ++i) {
      const int64_t bl0 = parts[i].r0 >> p.rbshift;
      const int64_t bl1 = ((int64_t)parts[i].r1 + (1ll << p.rbshift) - 1) >> p.rbshift;
      for (int64_t b = bl0; b < bl1 && b < p.nblk; ++b) mp[b] = (int32_t)(i - poff[pos]);
    }
  }
}

// One workgroup takes a strided share of one cut column's B entries and
// counts, per part, in LDS: the counting pass then adds its counts to bcnt,
// the filling pass reserves a range of each part's bucket (one atomic per
// part and workgroup) and walks its B entries again to fill the ranges.
// Columns with more than kBucketLds parts use global atomics per entry.
constexpr int kBucketLds = 4096;

template <bool FILL>
__global__ void __launch_bounds__(256) k_bucket(Operand B, ProdSrc S, PartCfg p, const int32_t* list,
                                                const int64_t* np, const int64_t* poff, int64_t multi_begin,
                                                int64_t multi_end, const Part* parts, const int32_t* map,
                                                unsigned* bcnt, const int64_t* boff, unsigned* bfill,
                                                int32_t* qlist, int64_t qcap, unsigned* err) {
  __shared__ unsigned s_cnt[kBucketLds];
  __shared__ int64_t s_base[FILL ? kBucketLds : 1];
  for (int64_t pos = multi_begin + blockIdx.y; pos < multi_end; pos += gridDim.y) {
    const int64_t npp = np[pos];
    if (npp <= 1) continue;
    const int32_t t = list[pos];
    const int64_t cb0 = slot_begin(B, t), cb1 = slot_begin(B, t + 1);
    const int64_t pbeg = poff[pos];
    const int32_t* mp = map + (pos - multi_begin) * p.nblk;
    const bool local = npp <= kBucketLds;
    // calls f(j) for every part j of the column that B entry q reaches
    auto reach = [&](int64_t q, auto&& f) {
      const int64_t a0 = S.a0[q];
      const int32_t alen = S.alen[q];
      const int32_t sid = S.splits ? S.split[q] : -1;
      if (sid >= 0 && alen > 2 * npp) {  // long A column: probe each part through the split table
        const int32_t* sp = S.splits + (int64_t)sid * S.sstride;
        for (int64_t j = 0; j < npp; ++j) {
          const Part& pj = parts[pbeg + j];
          const int32_t e0 = sp[pj.r0 >> S.rbshift];
          const int32_t e1 = sp[pj.r1 >= S.m ? S.sstride - 1 : (pj.r1 >> S.rbshift)];
          if (e1 > e0) f(j);
        }
      } else {  // short A column: walk its rows (sorted, so its parts come in order)
        int32_t last = -1;
        for (int32_t e = 0; e < alen; ++e) {
          const int32_t j = mp[S.air[a0 + e] >> S.rbshift];
          if (j >= 0 && j != last) {
            f(j);
            last = j;
          }
        }
      }
    };
    const int64_t q0 = cb0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t qs = (int64_t)gridDim.x * blockDim.x;
    if (!local) {  // uniform for the workgroup
      for (int64_t q = q0; q < cb1; q += qs)
        reach(q, [&](int64_t j) {
          if (FILL) {
            const int64_t at = boff[pbeg + j] + atomicAdd(&bfill[pbeg + j], 1u);
            if (at < qcap)
              qlist[at] = (int32_t)q;
            else
              atomicOr(err, 32u);
          } else {
            atomicAdd(&bcnt[pbeg + j], 1u);
          }
        });
      continue;
    }
    for (int64_t j = threadIdx.x; j < npp; j += blockDim.x) s_cnt[j] = 0;
    __syncthreads();
    for (int64_t q = q0; q < cb1; q += qs) reach(q, [&](int64_t j) { atomicAdd(&s_cnt[j], 1u); });
    __syncthreads();
    for (int64_t j = threadIdx.x; j < npp; j += blockDim.x) {
      const unsigned c = s_cnt[j];
      if (!FILL) {
        if (c) atomicAdd(&bcnt[pbeg + j], c);
      } else {
        s_base[j] = c ? boff[pbeg + j] + atomicAdd(&bfill[pbeg + j], c) : 0;
        s_cnt[j] = 0;
      }
    }
    __syncthreads();
    if (FILL) {
      for (int64_t q = q0; q < cb1; q += qs)
        reach(q, [&](int64_t j) {
          const int64_t at = s_base[j] + atomicAdd(&s_cnt[j], 1u);
          if (at < qcap)
            qlist[at] = (int32_t)q;
          else
            atomicOr(err, 32u);
        });
      __syncthreads();
    }
  }
}

__global__ void k_bucket_parts(const int64_t* np, const int64_t* poff, int64_t multi_begin, int64_t multi_end,
                               const unsigned* bcnt, const int64_t* boff, Part* parts) {
  for (int64_t pos = multi_begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pos < multi_end;
       pos += (int64_t)gridDim.x * blockDim.x) {
    if (np[pos] <= 1) continue;
    for (int64_t i = poff[pos]; i < poff[pos + 1]; ++i) {
      parts[i].b0 = boff[i];
      parts[i].nb = (int32_t)bcnt[i];
      parts[i].mode |= 2;
    }
  }
}

struct LoadBucket {
  const unsigned* p;
  __device__ int64_t operator()(int64_t i) const { return (int64_t)p[i]; }
};

// ------------------------------------------------------------------ numeric: parts
template <typename T>
__device__ __forceinline__ void block_bitonic_sort(uint64_t* a, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < (n2 >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (j - 1));
        const int hi = lo + j;
        const bool asc = (lo & k) == 0;
        const uint64_t x = a[lo], y = a[hi];
        if ((x > y) == asc) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// One workgroup per part (dynamic work queue).  Bitmap mode: mark rows,
// popcount prefix gives each row its rank = output position, accumulate
// values by rank, write rows and values in order.  Hash mode: accumulate
// into an open-addressing table, then sort (row, slot) keys.
template <int SR, typename T, int QC, bool OFF32>
__global__ void __launch_bounds__(1024) k_numeric_parts(Operand A, Operand B, ProdSrc S,
                                                        const int64_t* mults,
                                                        const int64_t* cnt, const Part* parts, const int64_t* qoff,
                                                        int nq, int nhome, unsigned long long* qctr,
                                                        const uint64_t* gbm, int64_t gbm_words,
                                                        const int32_t* qlist, int32_t* cir, T* cnum, unsigned* err) {
  using SR_ = Semiring<SR, T>;
  constexpr bool kVal = SR != SPX_OR_AND;
  constexpr int kPartBatch = 4;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int64_t s_pi;
  __shared__ int s_nbat;
  __shared__ Part s_batch[kPartBatch];
  __shared__ int64_t red[1024 / kWave + 1];
  __shared__ unsigned s_ctr;
  __shared__ RangeLdsT<QC> s_rng;
  const T* an = (const T*)A.num;
  const T* bn = (const T*)B.num;
  // work queues: queue k holds parts [qoff[k], qoff[k+1]); a workgroup
  // starts with its home queue (blockIdx.x % nhome: workgroups are placed on
  // the XCDs round robin, so one queue's rows of A stay in one L2), then
  // takes the shared queue nq-1, then helps the others.
  const int home = nhome > 1 ? (int)(blockIdx.x % nhome) : 0;
  // A ticket is a batch of up to kPartBatch consecutive parts (often of one
  // column), whose descriptors are loaded together.
  int qi = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      int64_t got = -1;
      int nbat = 0;
      while (qi < nq) {
        const int q = qi == 0 ? home : (qi == 1 ? nq - 1 : (home + qi - 1) % (nq - 1));
        const int64_t first = qoff[q] + (int64_t)atomicAdd(&qctr[q], (unsigned long long)kPartBatch);
        if (first < qoff[q + 1]) {
          got = first;
          nbat = (int)(qoff[q + 1] - first < kPartBatch ? qoff[q + 1] - first : kPartBatch);
          break;
        }
        ++qi;
      }
      s_pi = got;
      s_nbat = nbat;
    }
    __syncthreads();
    const int64_t pfirst = s_pi;
    const int nbat = s_nbat;
    if (pfirst < 0) break;
    if ((int)threadIdx.x < nbat) s_batch[threadIdx.x] = parts[pfirst + threadIdx.x];
    __syncthreads();
    for (int bi = 0; bi < nbat; ++bi) {
    const Part P = s_batch[bi];
    const int64_t b0 = P.b0, b1 = P.b0 + P.nb;
    const int32_t* qx = (P.mode & 2) ? qlist : nullptr;  // a bucketed part visits only its bucket
    const int64_t span = (int64_t)P.r1 - P.r0;
    const bool full = (P.r0 == 0 && P.r1 == (int32_t)A.m);
    // products in this part ~ mults * c / cnt
    const int c = P.c;
    if ((P.mode & 1) == 0) {
      const int W = (int)((span + 63) >> 6);
      uint64_t* bm = (uint64_t*)lds;
      uint16_t* pre = (uint16_t*)(bm + W);
      T* vals = (T*)(lds + W * 8 + ((W * 2 + 7) & ~7));
      // the row set: the count phase's stored bitmap, else marked here
      const bool stored = gbm != nullptr && P.bmi >= 0;
      if (stored) {
        const uint64_t* g = gbm + (int64_t)P.bmi * gbm_words + (P.r0 >> 6);
        for (int i0 = threadIdx.x; i0 < W; i0 += 4 * blockDim.x) {  // 4 loads in flight per thread
          uint64_t v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int i = i0 + k * (int)blockDim.x;
            v[k] = i < W ? g[i] : 0ull;
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int i = i0 + k * (int)blockDim.x;
            if (i < W) bm[i] = v[k];
          }
        }
      } else {
        for (int i = threadIdx.x; i < W; i += blockDim.x) bm[i] = 0;
      }
      if constexpr (kVal)
        for (int i = threadIdx.x; i < c; i += blockDim.x) vals[i] = SR_::ident();
      __syncthreads();
      if (!stored) {
        block_products<8, T, false, SR_::kUsesB, false, true, OFF32>(S, an, bn, b0, b1, P.r0, P.r1, full, s_rng, red, qx,
                                                  each_product<8>([&](int32_t r, T, T) {
          const uint32_t d = (uint32_t)(r - P.r0);
          atomicOr((unsigned long long*)&bm[d >> 6], 1ull << (d & 63));
        }));
        __syncthreads();
      }
      // exclusive popcount prefix per word
      const int per = (W + blockDim.x - 1) / blockDim.x;
      const int w0 = threadIdx.x * per;
      const int w1 = w0 + per < W ? w0 + per : W;
      int64_t s = 0;
      for (int i = w0; i < w1; ++i) s += __popcll(bm[i]);
      int64_t tot;
      int64_t run = block_excl_scan1(s, red, &tot);
      for (int i = w0; i < w1; ++i) {
        pre[i] = (uint16_t)run;
        run += __popcll(bm[i]);
      }
      if (threadIdx.x == 0 && tot != c) atomicOr(err, 8u);
      __syncthreads();
      if constexpr (kVal) {
        // rank of each product's row: all bitmap words first, then the adds
        auto acc = [&](const int32_t (&r)[8], const T (&a)[8], const T (&bv)[8]) {
          uint64_t w[8];
          int pr[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int wi = r[u] >= 0 ? (int)((uint32_t)(r[u] - P.r0) >> 6) : 0;
            w[u] = bm[wi];
            pr[u] = pre[wi];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (r[u] < 0) continue;
            const uint32_t d = (uint32_t)(r[u] - P.r0);
            const int rank = pr[u] + __popcll(w[u] & ((1ull << (d & 63)) - 1ull));
            if (rank < c) SR_::lds_acc(&vals[rank], SR_::mul(a[u], bv[u]));
          }
        };
        if (!stored && b1 - b0 <= (int64_t)(blockDim.x < QC ? blockDim.x : QC))
          block_products<8, T, SR_::kUsesA, SR_::kUsesB, true, true, OFF32>(S, an, bn, b0, b1, P.r0, P.r1, full, s_rng, red, qx, acc);
        else
          block_products<8, T, SR_::kUsesA, SR_::kUsesB, false, true, OFF32>(S, an, bn, b0, b1, P.r0, P.r1, full, s_rng, red, qx, acc);
        __syncthreads();
        // C is written once, coalesced: streaming stores keep the L2 for A's gathers
        // (a part's scattered hash-mode writes stay ordinary: streamed partial lines
        // cost more than they save)
        for (int i = threadIdx.x; i < c; i += blockDim.x) __builtin_nontemporal_store(vals[i], &cnum[P.off + i]);
        __syncthreads();
      }
      // rows in rank order: staged in the value area, then written coalesced
      int32_t* rows = (int32_t*)vals;
      for (int i = w0; i < w1; ++i) {
        uint64_t word = bm[i];
        int rk = pre[i];
        while (word) {
          const int bit = __ffsll((long long)word) - 1;
          word &= word - 1;
          if (rk < c) rows[rk] = P.r0 + i * 64 + bit;
          ++rk;
        }
      }
      __syncthreads();
      for (int i = threadIdx.x; i < c; i += blockDim.x) __builtin_nontemporal_store(rows[i], &cir[P.off + i]);
      __syncthreads();
    } else {
      int p2 = 64;
      while (p2 < c) p2 <<= 1;
      const uint32_t Sz = 2u * p2;
      const int log2s = 31 - __clz(Sz);
      uint32_t* keys = (uint32_t*)lds;
      T* vals = (T*)(lds + Sz * 4);
      unsigned char* tail = lds + Sz * 4 + ((Sz * sizeof(T) * (kVal ? 1 : 0) + 7) & ~7u);
      // row ranks by a two-level bitmap (spans up to kRankSpan rows): level 1
      // marks the nonempty 64-row groups, level 2 holds one word per nonempty
      // group; popcount prefixes of both give each row its rank.  Longer spans
      // sort (row, slot) keys instead.
      const bool ranked = span <= kRankSpan;
      const int n1 = (int)((span + 4095) >> 12);
      uint64_t* l2w = (uint64_t*)tail;
      uint16_t* l2p = (uint16_t*)(tail + p2 * 8);
      uint64_t* l1w = (uint64_t*)(tail + p2 * 10);
      uint16_t* l1p = (uint16_t*)(tail + p2 * 10 + (kRankSpan >> 9));
      uint64_t* sortb = (uint64_t*)tail;
      for (uint32_t i = threadIdx.x; i < Sz; i += blockDim.x) {
        keys[i] = 0xffffffffu;
        if constexpr (kVal) vals[i] = SR_::ident();
      }
      if (ranked) {
        for (int i = threadIdx.x; i < p2; i += blockDim.x) l2w[i] = 0;
        for (int i = threadIdx.x; i < n1; i += blockDim.x) l1w[i] = 0;
      }
      if (threadIdx.x == 0) s_ctr = 0;
      __syncthreads();
      block_products<4, T, SR_::kUsesA, SR_::kUsesB, false, false, OFF32>(S, an, bn, b0, b1, P.r0, P.r1, full, s_rng, red, qx,
                                                     each_product<4>([&](int32_t r, T a, T bv) {
        if (r < 0) return;
        uint32_t h = hash_row(r, log2s);
        for (uint32_t probe = 0; probe < Sz; ++probe) {
          const uint32_t old = atomicCAS(&keys[h], 0xffffffffu, (uint32_t)r);
          if (old == 0xffffffffu || old == (uint32_t)r) {
            if constexpr (kVal) SR_::lds_acc(&vals[h], SR_::mul(a, bv));
            return;
          }
          h = (h + 1) & (Sz - 1);
        }
        atomicOr(err, 16u);
      }));
      __syncthreads();
      if (ranked) {
        // level 1: nonempty groups of 64 rows
        for (uint32_t i = threadIdx.x; i < Sz; i += blockDim.x) {
          const uint32_t key = keys[i];
          if (key != 0xffffffffu) {
            const uint32_t g = (key - (uint32_t)P.r0) >> 6;
            atomicOr((unsigned long long*)&l1w[g >> 6], 1ull << (g & 63));
          }
        }
        __syncthreads();
        {
          const int per = (n1 + (int)blockDim.x - 1) / (int)blockDim.x;
          const int w0 = threadIdx.x * per, w1 = w0 + per < n1 ? w0 + per : n1;
          int64_t sum = 0;
          for (int w = w0; w < w1; ++w) sum += __popcll(l1w[w]);
          int64_t ng;
          int64_t run = block_excl_scan1(sum, red, &ng);
          for (int w = w0; w < w1; ++w) {
            l1p[w] = (uint16_t)run;
            run += __popcll(l1w[w]);
          }
        }
        __syncthreads();
        // level 2: the rows of each nonempty group
        for (uint32_t i = threadIdx.x; i < Sz; i += blockDim.x) {
          const uint32_t key = keys[i];
          if (key != 0xffffffffu) {
            const uint32_t d = key - (uint32_t)P.r0, g = d >> 6;
            const int gi = l1p[g >> 6] + __popcll(l1w[g >> 6] & ((1ull << (g & 63)) - 1ull));
            if (gi < p2) atomicOr((unsigned long long*)&l2w[gi], 1ull << (d & 63));
          }
        }
        __syncthreads();
        int64_t found;
        {
          const int per = (p2 + (int)blockDim.x - 1) / (int)blockDim.x;
          const int w0 = threadIdx.x * per, w1 = w0 + per < p2 ? w0 + per : p2;
          int64_t sum = 0;
          for (int w = w0; w < w1; ++w) sum += __popcll(l2w[w]);
          int64_t run = block_excl_scan1(sum, red, &found);
          for (int w = w0; w < w1; ++w) {
            l2p[w] = (uint16_t)run;
            run += __popcll(l2w[w]);
          }
        }
        __syncthreads();
        if (threadIdx.x == 0 && found != c) atomicOr(err, 32u);
        // rank = output position
        for (uint32_t i = threadIdx.x; i < Sz; i += blockDim.x) {
          const uint32_t key = keys[i];
          if (key != 0xffffffffu) {
            const uint32_t d = key - (uint32_t)P.r0, g = d >> 6;
            const int gi = l1p[g >> 6] + __popcll(l1w[g >> 6] & ((1ull << (g & 63)) - 1ull));
            if (gi < p2) {
              const int rank = l2p[gi] + __popcll(l2w[gi] & ((1ull << (d & 63)) - 1ull));
              if (rank < c) {
                cir[P.off + rank] = (int32_t)key;
                if constexpr (kVal) cnum[P.off + rank] = vals[i];
              }
            }
          }
        }
      } else {
        for (uint32_t i = threadIdx.x; i < Sz; i += blockDim.x) {
          const uint32_t key = keys[i];
          if (key != 0xffffffffu) {
            const unsigned p = atomicAdd(&s_ctr, 1u);
            if ((int)p < p2) sortb[p] = ((uint64_t)key << 32) | i;
          }
        }
        __syncthreads();
        const int found = (int)s_ctr;
        if (threadIdx.x == 0 && found != c) atomicOr(err, 32u);
        for (int i = found + threadIdx.x; i < p2; i += blockDim.x) sortb[i] = ~0ull;
        __syncthreads();
        block_bitonic_sort<T>(sortb, p2);
        for (int i = threadIdx.x; i < c; i += blockDim.x) {
          const uint64_t k = sortb[i];
          cir[P.off + i] = (int32_t)(k >> 32);
          if constexpr (kVal) cnum[P.off + i] = vals[k & 0xffffffffu];
        }
      }
      __syncthreads();
    }
    }
  }
}

// ------------------------------------------------------------------ output pointers
__global__ void k_nonzero_flags_count(const int64_t* cnt, int64_t n, unsigned long long* nz) {
  int64_t s = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) s += cnt[i] > 0;
  s = wave_sum(s);
  if (lane_id() == 0 && s) atomicAdd(nz, (unsigned long long)s);
}

// CSC output: cp[j] = start of column j.  For a DCSC B, column j's start is
// the offset of the first slot whose column id is >= j.
__global__ void k_write_csc_cp(Operand B, const int64_t* off, int64_t nslots, int64_t n, void* cp, int32_t ptr_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n; j += stride) {
    int64_t t = j;
    if (B.fmt == SPX_DCSC) {
      int64_t lo = 0, hi = nslots;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)B.jc[mid] < j)
          lo = mid + 1;
        else
          hi = mid;
      }
      t = lo;
    }
    store_ptr(cp, ptr_t, j, off[t]);
  }
}

// DCSC output: nonempty slot t becomes entry zoff[t] of jc / cp.
__global__ void k_write_dcsc(Operand B, const int64_t* cnt, const int64_t* off, const int64_t* zoff, int64_t nslots,
                             int32_t* jc, void* cp, int32_t ptr_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nslots; t += stride) {
    if (cnt[t] > 0) {
      const int64_t u = zoff[t];
      jc[u] = (int32_t)slot_col(B, t);
      store_ptr(cp, ptr_t, u, off[t]);
    }
    if (t == nslots - 1) store_ptr(cp, ptr_t, zoff[nslots], off[nslots]);
  }
}

// Sum of the exact counts of the columns in bin `bin`.
__global__ void k_bin_sum(const int32_t* list, const int64_t* binoff, int bin, const int64_t* cnt,
                          unsigned long long* out) {
  const int64_t beg = binoff[bin], end = binoff[bin + 1];
  int64_t s = 0;
  for (int64_t p = beg + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < end; p += (int64_t)gridDim.x * blockDim.x)
    s += cnt[list[p]];
  s = wave_sum(s);
  if (lane_id() == 0 && s) atomicAdd(out, (unsigned long long)s);
}

__global__ void k_parts_sum(const Part* parts, int64_t n, unsigned long long* out) {
  int64_t s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += parts[i].c;
  s = wave_sum(s);
  if (lane_id() == 0 && s) atomicAdd(out, (unsigned long long)s);
}

// Counting sort of the multi-part list by row slice (work queue).
__global__ void k_part_hist(const Part* parts, int64_t n, unsigned long long* hist) {
  __shared__ unsigned h[66];
  for (int i = threadIdx.x; i < 66; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&h[parts[i].slice], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < 66; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// Exclusive offsets of nb bins, written to cursor and to qoff (+ qoff[nb]).
__global__ void k_hist_offsets(unsigned long long* hist, int64_t nb, int64_t base, int64_t* qoff) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const unsigned long long c = hist[b];
      hist[b] = run;
      qoff[b] = base + (int64_t)run;
      run += c;
    }
    qoff[nb] = base + (int64_t)run;
  }
}

// Per block: rank inside the block by LDS atomics, one global atomic per bin.
__global__ void k_part_scatter(const Part* in, int64_t n, unsigned long long* cursor, Part* out) {
  __shared__ unsigned h[66];
  __shared__ unsigned long long base[66];
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < n; t0 += (int64_t)gridDim.x * blockDim.x) {
    for (int i = threadIdx.x; i < 66; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t i = t0 + threadIdx.x;
    Part p{};
    unsigned rk = 0;
    if (i < n) {
      p = in[i];
      rk = atomicAdd(&h[p.slice], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 66; b += blockDim.x)
      if (h[b]) base[b] = atomicAdd(&cursor[b], (unsigned long long)h[b]);
    __syncthreads();
    if (i < n) out[base[p.slice] + rk] = p;
    __syncthreads();
  }
}

struct NonzeroFlag {
  const int64_t* cnt;
  __device__ int64_t operator()(int64_t i) const { return cnt[i] > 0 ? 1 : 0; }
};

}  // namespace spx

// ==================================================================== host
using namespace spx;

namespace spx {

struct Summary {
  unsigned long long mults;
  unsigned long long nnz_tiny;
  unsigned long long nnz_multi;
  unsigned long long setup;      // sum over cut columns of (B entries x parts)
  unsigned long long cut_mults;  // multiplications of the cut columns
  unsigned err;
  unsigned pad;
};

enum { kEvPlan0, kEvPlan1, kEvExec0, kEvMulti, kEvParts, kEvTiny, kEvPtr, kNumEv };

struct GemmPlan : spx_plan {
  explicit GemmPlan(const spx_ctx* c) : spx_plan(c, kPlanGemm) {
    if (c && c->profile) {
      profile = true;
      for (auto& e : ev) (void)hipEventCreate(&e);
    }
  }
  ~GemmPlan() override {
    if (profile)
      for (auto& e : ev) (void)hipEventDestroy(e);
  }
  void mark(int i, hipStream_t st) {
    if (profile) (void)hipEventRecord(ev[i], st);
  }
  bool profile = false;
  bool ran_parts = false, ran_tiny = false;
  hipEvent_t ev[kNumEv] = {};
  Operand A{}, B{};
  int32_t sr = 0, vt = 0, c_fmt = 0;
  spx_tuning tune{};
  int64_t nslots = 0, nnz = 0, nzc = 0, mults = 0, nparts = 0, psplit = 0, nnz_tiny = 0, nnz_multi = 0;
  int64_t binoff_h[kNumBins + 1] = {};
  int64_t* bq_a0 = nullptr;
  int32_t* bq_alen = nullptr;
  int32_t* bq_split = nullptr;
  int32_t* splits = nullptr;
  ProdSrc src{};
  int64_t* aux = nullptr;
  int64_t* mults_d = nullptr;
  int64_t* cnt = nullptr;
  int64_t* off = nullptr;
  int64_t* zoff = nullptr;
  int32_t* list = nullptr;
  int64_t* binoff = nullptr;
  Part* parts = nullptr;
  int64_t* qoff_multi = nullptr;
  unsigned long long* qctr = nullptr;
  int64_t* qoff_single = nullptr;
  int32_t nq_multi = 1, nslice = 1, nslice_req = 1;
  Summary* sum = nullptr;
  int64_t L = 0, L_single = 0;
  bool wide = false;  // the multi-part launch uses the wide range list
  int32_t* qlist = nullptr;  // B entries of the parts of bucketed columns, grouped by part
  uint64_t* gbm = nullptr;  // stored row bitmaps of the bitmap-counted columns
  int64_t gbm_words = 0;    // 64-bit words per stored bitmap
};

int check_mat(const spx_mat* X, const char* name) {
  if (!X) return fail(SPX_EINVAL, std::string(name) + " is NULL");
  if (X->m < 0 || X->n < 0 || X->nnz < 0 || X->m >= (1ll << 31) || X->n >= (1ll << 31))
    return fail(SPX_EINVAL, std::string(name) + ": bad dimensions");
  if (X->fmt != SPX_CSC && X->fmt != SPX_DCSC) return fail(SPX_EINVAL, std::string(name) + ": bad format");
  if (X->ptr_t != SPX_PTR_I32 && X->ptr_t != SPX_PTR_I64) return fail(SPX_EINVAL, std::string(name) + ": bad ptr_t");
  if (X->val_t < SPX_VAL_F32 || X->val_t > SPX_VAL_BOOL) return fail(SPX_EINVAL, std::string(name) + ": bad val_t");
  if (X->ptr_t == SPX_PTR_I32 && X->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, std::string(name) + ": nnz needs I64 pointers");
  if (X->fmt == SPX_DCSC && (X->nzc < 0 || X->nzc > X->n || (X->nzc > 0 && !X->jc)))
    return fail(SPX_EINVAL, std::string(name) + ": bad DCSC nzc/jc");
  if (!X->cp) return fail(SPX_EINVAL, std::string(name) + ": cp is NULL");
  if (X->nnz > 0 && !X->ir) return fail(SPX_EINVAL, std::string(name) + ": ir is NULL");
  if (X->nnz > 0 && X->val_t != SPX_VAL_BOOL && !X->num) return fail(SPX_EINVAL, std::string(name) + ": num is NULL");
  return SPX_OK;
}

int build_aux(const Operand& X, Scratch& scr, hipStream_t st, int64_t** aux, int64_t* chunk) {
  *aux = nullptr;
  *chunk = 1;
  if (X.fmt != SPX_DCSC) return SPX_OK;
  *chunk = std::max<int64_t>(1, ceil_div(std::max<int64_t>(X.n, 1), std::max<int64_t>(X.nzc, 1)));
  const int64_t naux = ceil_div(std::max<int64_t>(X.n, 1), *chunk);
  SPX_TRY(scr.get_n(naux + 1, aux));
  k_build_aux<<<grid_for(naux + 1, 256), 256, 0, st>>>(X.jc, X.nzc, *chunk, naux, *aux);
  SPX_HIP(hipGetLastError());
  return SPX_OK;
}

// Waits for the stream and reads the plan's summary together with the
// given extra device words (one read-back launch).
int summary_sync(GemmPlan* P, hipStream_t st, Summary* host, std::initializer_list<DevWord> extra = {},
                 int64_t* extra_out = nullptr) {
  static_assert(sizeof(Summary) == 6 * sizeof(int64_t), "the summary is read as six words");
  DevWord w[kMaxReadRanges];
  int n = 0, nx = 0;
  for (const DevWord& d : extra) {
    w[n++] = d;
    nx += d.count;
  }
  w[n++] = DevWord{P->sum, 8, 6};
  int64_t out[kMaxReadWords];
  SPX_TRY(read_device_words(st, w, n, out));
  for (int i = 0; i < nx; ++i) extra_out[i] = out[i];
  std::memcpy(host, out + nx, sizeof(Summary));
  return SPX_OK;
}

}  // namespace spx

extern "C" void spx_default_tuning(spx_tuning* t) {
  std::memset(t, 0, sizeof(*t));
  t->tiny_max = 64;
  t->hash_count_max = 1 << 13;
  t->single_part_max = 1024;
  t->part_lds_bytes = 72 * 1024;
  t->count_threads = 256;
  t->bitmap_threads = 512;
  t->part_threads = 512;
  t->single_threads = 256;
  t->bitmap_chunk_log2 = 0;
  t->xcd_slices = 1;
  t->bitmap_store_mb = 32768;
}

template <int SR, typename T>
static int launch_numeric(GemmPlan* P, spx_mat* C, hipStream_t st) {
  int32_t* cir = C->ir;
  T* cnum = (T*)C->num;
  unsigned* err = &P->sum->err;
  const int cus = device_cu_count();
  // parts of multi-part columns [0, psplit), single-part columns [psplit, nparts)
  if (P->nparts > 0) SPX_TRY(fill_i64((int64_t*)P->qctr, P->nq_multi + 2, 0, st));
  for (int r = 0; r < 2; ++r) {
    const int64_t n0 = r == 0 ? 0 : P->psplit, n1 = r == 0 ? P->psplit : P->nparts;
    if (n1 <= n0) continue;
    const int blk = r == 0 ? P->tune.part_threads : P->tune.single_threads;
    const int64_t L = r == 0 ? P->L : P->L_single;
    const int per_cu = (int)std::max<int64_t>(1, std::min<int64_t>((160 * 1024) / (L + 8192), 2048 / blk));
    int64_t grid = std::min<int64_t>(n1 - n0, (int64_t)cus * per_cu);
    if (r == 0 && P->nslice > 1) grid = std::max<int64_t>(P->nslice, grid / P->nslice * P->nslice);
    const int64_t* qoff = r == 0 ? P->qoff_multi : P->qoff_single;
    const int nq = r == 0 ? P->nq_multi : 1;
    unsigned long long* qctr = r == 0 ? P->qctr : P->qctr + P->nq_multi;
    if (r == 0 && P->wide)
      hipLaunchKernelGGL((k_numeric_parts<SR, T, kQChunkWide, false>), dim3((unsigned)grid), dim3(blk), (size_t)L, st,
                         P->A, P->B, P->src, P->mults_d, P->cnt, P->parts, qoff, nq, P->nslice, qctr, P->gbm,
                         P->gbm_words, P->qlist, cir, cnum, err);
    else if (P->src.off32)  // A's positions fit 29 bits: gathers through 32-bit offsets
      hipLaunchKernelGGL((k_numeric_parts<SR, T, kQChunk, true>), dim3((unsigned)grid), dim3(blk), (size_t)L, st, P->A,
                         P->B, P->src, P->mults_d, P->cnt, P->parts, qoff, nq, r == 0 ? P->nslice : 1, qctr, P->gbm,
                         P->gbm_words, P->qlist, cir, cnum, err);
    else
      hipLaunchKernelGGL((k_numeric_parts<SR, T, kQChunk, false>), dim3((unsigned)grid), dim3(blk), (size_t)L, st, P->A,
                         P->B, P->src, P->mults_d, P->cnt, P->parts, qoff, nq, r == 0 ? P->nslice : 1, qctr, P->gbm,
                         P->gbm_words, P->qlist, cir, cnum, err);
    SPX_HIP(hipGetLastError());
    if (r == 0) P->mark(kEvMulti, st);
  }
  if (P->psplit == 0) P->mark(kEvMulti, st);
  P->mark(kEvParts, st);
  const int64_t ntiny = P->binoff_h[kBinTiny + 1] - P->binoff_h[kBinTiny];
  if (ntiny > 0) {
    hipLaunchKernelGGL((k_tiny<SR, T, false>), dim3(grid_for(ntiny, 8, (int64_t)cus * 16)), dim3(256), 0, st, P->A,
                       P->B, P->bq_a0, P->bq_alen, P->mults_d, P->list, P->binoff, P->cnt, P->off, cir, cnum);
    SPX_HIP(hipGetLastError());
  }
  P->mark(kEvTiny, st);
  return SPX_OK;
}

static int dispatch_numeric(GemmPlan* P, spx_mat* C, hipStream_t st) {
#define SPX_CASE(SRV, VTV, TY) \
  if (P->sr == SRV && P->vt == VTV) return launch_numeric<SRV, TY>(P, C, st);
  SPX_CASE(SPX_PLUS_TIMES, SPX_VAL_F32, float)
  SPX_CASE(SPX_PLUS_TIMES, SPX_VAL_F64, double)
  SPX_CASE(SPX_PLUS_TIMES, SPX_VAL_I64, int64_t)
  SPX_CASE(SPX_MIN_PLUS, SPX_VAL_F32, float)
  SPX_CASE(SPX_MIN_PLUS, SPX_VAL_F64, double)
  SPX_CASE(SPX_MIN_PLUS, SPX_VAL_I64, int64_t)
  SPX_CASE(SPX_SELECT2ND, SPX_VAL_F32, float)
  SPX_CASE(SPX_SELECT2ND, SPX_VAL_F64, double)
  SPX_CASE(SPX_SELECT2ND, SPX_VAL_I64, int64_t)
  SPX_CASE(SPX_SELECT1ST, SPX_VAL_F32, float)
  SPX_CASE(SPX_SELECT1ST, SPX_VAL_F64, double)
  SPX_CASE(SPX_SELECT1ST, SPX_VAL_I64, int64_t)
  if (P->sr == SPX_OR_AND || P->vt == SPX_VAL_BOOL) return launch_numeric<SPX_OR_AND, float>(P, C, st);
#undef SPX_CASE
  return fail(SPX_EUNSUPPORTED, "semiring / value type combination not provided");
}

// Result value type of a product, or -1 when the combination is not provided.
static int result_type(int32_t sr, const spx_mat* A, const spx_mat* B) {
  switch (sr) {
    case SPX_PLUS_TIMES:
    case SPX_MIN_PLUS:
      if (A->val_t != B->val_t || A->val_t == SPX_VAL_BOOL) return -1;
      return A->val_t;
    case SPX_SELECT2ND: return B->val_t;
    case SPX_SELECT1ST: return A->val_t;
    case SPX_OR_AND: return SPX_VAL_BOOL;
    default: return -1;
  }
}

extern "C" int spx_spgemm_plan(const spx_ctx* ctx, const spx_mat* A, const spx_mat* B, int32_t semiring,
                               int32_t c_fmt, const spx_tuning* tuning, spx_plan** plan, int64_t* nnz_c,
                               int64_t* nzc_c) {
  if (!plan) return fail(SPX_EINVAL, "plan is NULL");
  *plan = nullptr;
  SPX_TRY(check_mat(A, "A"));
  SPX_TRY(check_mat(B, "B"));
  if (A->n != B->m) return fail(SPX_EINVAL, "inner dimensions differ: A is m x k, B must be k x n");
  if (c_fmt != SPX_CSC && c_fmt != SPX_DCSC) return fail(SPX_EINVAL, "bad output format");
  const int vt = result_type(semiring, A, B);
  if (vt < 0) return fail(SPX_EUNSUPPORTED, "semiring / value type combination not provided");
  spx_tuning tune;
  spx_default_tuning(&tune);
  if (tuning) tune = *tuning;
  if (tune.tiny_max < 0 || tune.tiny_max > 64) return fail(SPX_EINVAL, "tiny_max must be in [0, 64]");
  if (tune.hash_count_max < tune.tiny_max || tune.hash_count_max > (1 << 14))
    return fail(SPX_EINVAL, "hash_count_max must be in [tiny_max, 16384]");
  if (tune.single_part_max < 64 || tune.single_part_max > 4096 || (tune.single_part_max & (tune.single_part_max - 1)))
    return fail(SPX_EINVAL, "single_part_max must be a power of two in [64, 4096]");
  if (tune.range_chunk != 0 && tune.range_chunk != kQChunk && tune.range_chunk != kQChunkWide)
    return fail(SPX_EINVAL, "range_chunk must be 0, 256 or 512");
  for (int th : {tune.count_threads, tune.bitmap_threads, tune.part_threads, tune.single_threads})
    if (th % 64 || th < 64 || th > 1024) return fail(SPX_EINVAL, "thread counts must be multiples of 64 in [64, 1024]");

  if (ctx && ctx->validate) {
    int32_t ok = 0;
    SPX_TRY(spx_check(ctx, A, &ok));
    if (!ok) return fail(SPX_EINVAL, "A is not canonical");
    SPX_TRY(spx_check(ctx, B, &ok));
    if (!ok) return fail(SPX_EINVAL, "B is not canonical");
  }
  auto* P = new GemmPlan(ctx);
  std::unique_ptr<GemmPlan> guard(P);
  hipStream_t st = stream_of(ctx);
  Scratch& scr = P->scratch;
  P->A = make_operand(A);
  P->B = make_operand(B);
  P->sr = semiring;
  P->vt = vt;
  P->c_fmt = c_fmt;
  P->tune = tune;
  const int sz = value_size(vt);
  const int64_t m = A->m;
  P->nslots = nslots_of(P->B);
  const int64_t nslots = P->nslots;
  const int cus = device_cu_count();

  // Row blocks: the largest power of two <= 2^14 such that one dense block
  // fits a part in bitmap mode.
  int64_t L = tune.part_lds_bytes;
  if (L > 160 * 1024 - 8192) L = 160 * 1024 - 8192;
  int rb = 14;
  while (rb > 6 && ((1ll << rb) * sz + ((1ll << rb) / 64) * 10 + 256) > L) --rb;
  if (((1ll << rb) * sz + ((1ll << rb) / 64) * 10 + 256) > L) return fail(SPX_EINVAL, "part_lds_bytes too small");
  P->L = L;
  int sp_log2 = 6;
  while ((1 << sp_log2) < tune.single_part_max) ++sp_log2;
  {
    const int64_t p2 = tune.single_part_max, S2 = 2 * p2;
    P->L_single = S2 * 4 + ((S2 * sz + 7) & ~7ll) + p2 * 10 + (kRankSpan >> 9) + (kRankSpan >> 11) + 64;
    if (P->L_single > 160 * 1024 - 8192) return fail(SPX_EINVAL, "single_part_max too large for LDS");
  }
  const int64_t nblk = std::max<int64_t>(1, ceil_div(m, 1ll << rb));
  P->nslice_req = std::max(1, std::min(tune.xcd_slices, 64));
  P->mark(kEvPlan0, st);

  unsigned long long *bincount = nullptr, *binfill = nullptr, *nlong = nullptr;
  int32_t* longs = nullptr;  // slots with more than kLongSlot B entries
  SPX_TRY(scr.get_many({Scratch::part(&P->sum, 1), Scratch::part(&P->bq_a0, B->nnz),
                        Scratch::part(&P->bq_alen, B->nnz), Scratch::part(&P->bq_split, B->nnz),
                        Scratch::part(&P->mults_d, nslots), Scratch::part(&P->cnt, nslots),
                        Scratch::part(&P->off, nslots + 1), Scratch::part(&P->zoff, nslots + 1),
                        Scratch::part(&P->list, nslots), Scratch::part(&P->binoff, kNumBins + 1),
                        Scratch::part(&bincount, kNumBins), Scratch::part(&binfill, kNumBins),
                        Scratch::part(&longs, std::max<int64_t>(nslots, 1)), Scratch::part(&nlong, 1)}));
  // bin offsets stay zero when there are no slots (k_bin_fill writes them otherwise)
  SPX_TRY(zero_words(st, {{P->sum, (int64_t)(sizeof(Summary) / 8)}, {bincount, kNumBins}, {binfill, kNumBins},
                          {P->cnt, std::max<int64_t>(nslots, 1)}, {nlong, 1}, {P->binoff, kNumBins + 1}}));
  unsigned* err = &P->sum->err;

  // AUX index for a DCSC A
  int64_t chunk = 1;
  SPX_TRY(build_aux(P->A, scr, st, &P->aux, &chunk));
  // split table of A's long columns
  const int64_t nslots_a = nslots_of(P->A);
  const int64_t split_cap = A->nnz / (kSplitMin + 1) + 1;
  const int32_t sstride = (int32_t)nblk + 1;
  int64_t* sid_off = nullptr;
  if (A->nnz > kSplitMin && nslots_a > 0) {
    int32_t* slot_of_split = nullptr;
    SPX_TRY(scr.get_n(nslots_a + 1, &sid_off));
    SPX_TRY(scr.get_n(split_cap, &slot_of_split));
    SPX_TRY(scr.get_n(split_cap * sstride, &P->splits));
    SPX_TRY(exclusive_scan(LongColumn{P->A}, nslots_a, sid_off, scr, st));
    k_split_rows<<<grid_for(nslots_a, 256, 65536), 256, 0, st>>>(P->A, nslots_a, sid_off, slot_of_split);
    SPX_HIP(hipGetLastError());
    k_split_fill<<<grid_for(split_cap * kWave, 256, (int64_t)cus * 32), 256, 0, st>>>(
        P->A, sid_off + nslots_a, split_cap, slot_of_split, P->splits, sstride, rb);
    SPX_HIP(hipGetLastError());
  }
  if (B->nnz > 0) {
    k_rowinfo<<<grid_for(B->nnz, 256, (int64_t)cus * 32), 256, 0, st>>>(P->A, P->B, P->aux, chunk, sid_off, P->bq_a0,
                                                                         P->bq_alen, P->bq_split, err);
    SPX_HIP(hipGetLastError());
  }
  P->src = ProdSrc{A->ir, P->bq_a0, P->bq_alen, P->bq_split, P->splits, sstride, rb, (int32_t)m,
                   (A->nnz < (1ll << 29) && !tune.force_off64) ? 1 : 0};
  BinCfg bc{tune.tiny_max, tune.hash_count_max};
  if (nslots > 0) {
    k_slot_mults<<<grid_for(nslots * 8, 256, (int64_t)cus * 16), 256, 0, st>>>(P->B, P->bq_alen, nslots, P->mults_d,
                                                                              &P->sum->mults, longs, nlong);
    SPX_HIP(hipGetLastError());
    k_slot_mults_long<<<(unsigned)cus * 4, 256, 0, st>>>(P->B, P->bq_alen, longs, nlong, P->mults_d, &P->sum->mults);
    SPX_HIP(hipGetLastError());
    k_bin_count<<<grid_for(nslots, 256, (int64_t)cus * 8), 256, 0, st>>>(P->mults_d, nslots, bc, bincount);
    SPX_HIP(hipGetLastError());
  }
  if (nslots > 0) {
    k_bin_fill<<<grid_for(ceil_div(nslots, kFillPer), 256, (int64_t)cus * 8), 256, 0, st>>>(
        P->mults_d, nslots, bc, bincount, P->binoff, binfill, P->list);
    SPX_HIP(hipGetLastError());
  }
  // sync 1: bin sizes and the total number of multiplications
  Summary hs{};
  static_assert(sizeof(P->binoff_h) == (kNumBins + 1) * sizeof(int64_t), "bin offsets are read as words");
  SPX_TRY(summary_sync(P, st, &hs, {{P->binoff, 8, kNumBins + 1}}, P->binoff_h));
  if (hs.err & 1u) return fail(SPX_EINVAL, "B has a row index outside A's columns");
  P->mults = (int64_t)hs.mults;
  const int64_t* bo = P->binoff_h;
  // columns with more than single_part_max products get row-block counts
  const int64_t multi_begin = bo[0], multi_end = bo[std::min(kBinHash0 + 14 - sp_log2, kBinTiny)];
  const int64_t nmulti = multi_end - multi_begin;
  uint32_t* blkcnt = nullptr;
  if (nmulti > 0) {
    if ((double)nmulti * (double)nblk * 4.0 > 8e9) return fail(SPX_EUNSUPPORTED, "row-block table too large");
    SPX_TRY(scr.get_n(nmulti * nblk, &blkcnt));
    SPX_TRY(fill_u32(blkcnt, nmulti * nblk, 0, st));
  }

  // exact counts
  const int64_t ntiny = bo[kBinTiny + 1] - bo[kBinTiny];
  if (ntiny > 0) {
    k_tiny<SPX_OR_AND, float, true><<<grid_for(ntiny, 8, (int64_t)cus * 16), 256, 0, st>>>(
        P->A, P->B, P->bq_a0, P->bq_alen, P->mults_d, P->list, P->binoff, P->cnt, nullptr, nullptr, nullptr);
    SPX_HIP(hipGetLastError());
  }
  for (int b = kBinHash0; b < kBinTiny; ++b) {
    const int64_t nb = bo[b + 1] - bo[b];
    if (nb == 0) continue;
    const int log2s = kHashLog2Max - (b - kBinHash0);
    const size_t lds = ((size_t)4 << log2s) + (nblk <= 1024 ? (size_t)nblk * 4 : 0);
    const int blk = log2s >= 15 ? 1024 : (log2s >= 13 ? std::max(tune.count_threads, 512) : tune.count_threads);
    const int per_cu = std::max<int>(1, (int)((160 * 1024) / (lds + 8192)));
    k_count_hash<<<(unsigned)std::min<int64_t>(nb, (int64_t)cus * per_cu), blk, lds, st>>>(
        P->B, P->src, P->mults_d, P->list, P->binoff, b, log2s, multi_end, rb, nblk, blkcnt, P->cnt, err);
    SPX_HIP(hipGetLastError());
  }
  const int64_t nbitmap = bo[kBinHash0] - bo[0];
  if (nbitmap > 0) {
    // bitmap chunks: a power of two of rows, a multiple of the row block;
    // 0 = one chunk per row slice
    int want = tune.bitmap_chunk_log2;
    if (want <= 0) {  // auto: one chunk per row slice, at most 2^18 rows (four workgroups per CU)
      want = 0;
      while ((1ll << want) < ceil_div(m, std::max(1, P->nslice_req))) ++want;
      want = std::min(want, 18);
    }
    int clog = std::max<int>(rb, std::min<int>(want, 20));
    while (clog > rb && (1ll << (clog - 1)) >= m) --clog;
    const int64_t nchunks = ceil_div(m, 1ll << clog);
    const size_t lds = ((size_t)1 << clog) / 8 + (((size_t)1 << clog) >> rb) * 4 + 16;
    const int per_cu = std::max<int>(1, std::min<int>((int)((160 * 1024) / (lds + 8192)), 2048 / tune.bitmap_threads));
    int64_t bgrid = std::min<int64_t>(nbitmap * nchunks, (int64_t)cus * per_cu);
    bgrid = std::max<int64_t>(nchunks, bgrid / nchunks * nchunks);
    unsigned long long* bqctr = nullptr;  // per-chunk column counters
    SPX_TRY(scr.get_n(nchunks, &bqctr));
    SPX_TRY(fill_i64((int64_t*)bqctr, nchunks, 0, st));
    // keep the bitmaps for the numeric phase when they fit the cap
    const int64_t words = ceil_div(m, 64);
    if (tune.bitmap_store_mb > 0 && (double)nbitmap * words * 8.0 <= (double)tune.bitmap_store_mb * 1048576.0) {
      if (scr.get_n(nbitmap * words, &P->gbm) == SPX_OK)
        P->gbm_words = words;
      else
        P->gbm = nullptr;  // not enough memory: recompute instead
    }
    k_count_bitmap<<<(unsigned)bgrid, tune.bitmap_threads, lds, st>>>(
        P->B, P->src, P->mults_d, P->list, P->binoff, m, clog, rb, nblk, blkcnt, (unsigned long long*)P->cnt,
        (uint32_t*)P->gbm, 2 * P->gbm_words, bqctr);
    SPX_HIP(hipGetLastError());
  }
  // column pointers and nonempty-column offsets
  SPX_TRY(exclusive_scan(LoadI64{P->cnt}, nslots, P->off, scr, st));
  SPX_TRY(exclusive_scan(NonzeroFlag{P->cnt}, nslots, P->zoff, scr, st));
  // parts of the non-tiny columns: list positions [0, bo[kBinTiny])
  const int64_t npos = bo[kBinTiny];
  int64_t *np = nullptr, *poff = nullptr;
  int nslice = std::max(1, std::min(tune.xcd_slices, 64));
  int64_t slice_blocks = ceil_div(nblk, nslice);
  nslice = (int)ceil_div(nblk, slice_blocks);
  if (nslice <= 1) slice_blocks = 0;
  P->nslice = nslice;
  PartCfg pc{L, m, sz, rb, nblk, slice_blocks, nslice, 0};
  PartCfg pcs{P->L_single, m, sz, rb, nblk, 0, nslice, 0};
  if (npos > 0) {
    SPX_TRY(scr.get_n(npos, &np));
    SPX_TRY(scr.get_n(npos + 1, &poff));
    k_parts<<<grid_for(npos, 256, (int64_t)cus * 16), 256, 0, st>>>(P->B, pc, pcs, P->list, npos, multi_begin, multi_end,
                                                                    P->gbm ? nbitmap : 0, P->cnt,
                                                                    P->off, blkcnt, np, nullptr, nullptr, P->mults_d,
                                                                    &P->sum->setup, err);
    SPX_HIP(hipGetLastError());
    SPX_TRY(exclusive_scan(LoadI64{np}, npos, poff, scr, st));
  }
  if (ntiny > 0) {
    k_bin_sum<<<grid_for(ntiny, 256, 1024), 256, 0, st>>>(P->list, P->binoff, kBinTiny, P->cnt, &P->sum->nnz_tiny);
    SPX_HIP(hipGetLastError());
  }
  // sync 2: sizes
  int64_t tail[4] = {0, 0, 0, 0};
  if (npos > 0)
    SPX_TRY(summary_sync(P, st, &hs, {{P->off + nslots, 8}, {P->zoff + nslots, 8}, {poff + npos, 8},
                                      {poff + multi_end, 8}}, tail));
  else
    SPX_TRY(summary_sync(P, st, &hs, {{P->off + nslots, 8}, {P->zoff + nslots, 8}}, tail));
  if (hs.err & 4u) return fail(SPX_EUNSUPPORTED, "a row block is too dense for the LDS budget");
  // Columns with many B entries per product (a tall-skinny right operand):
  // every part walks all of its column's B entries, so range set-ups
  // outnumber products.  Then the multi-part launch takes twice as many B
  // entries per set-up round, and its parts are re-cut for the LDS that the
  // larger range list leaves, if a dense row block still fits.
  const bool want_wide = tune.range_chunk == kQChunkWide ||
                         (tune.range_chunk == 0 && hs.cut_mults > 0 && 2 * hs.setup > hs.cut_mults);
  if (npos > 0 && want_wide) {
    const int64_t Lw = L - kWideExtraLds;
    if (((1ll << rb) * sz + ((1ll << rb) / 64) * 10 + 256) <= Lw) {
      P->wide = true;
      P->L = Lw;
      pc.L = Lw;
      SPX_TRY(fill_i64(reinterpret_cast<int64_t*>(&P->sum->setup), 2, 0, st));  // the cut columns may change
      k_parts<<<grid_for(npos, 256, (int64_t)cus * 16), 256, 0, st>>>(
          P->B, pc, pcs, P->list, npos, multi_begin, multi_end, P->gbm ? nbitmap : 0, P->cnt, P->off, blkcnt, np,
          nullptr, nullptr, P->mults_d, &P->sum->setup, err);
      SPX_HIP(hipGetLastError());
      SPX_TRY(exclusive_scan(LoadI64{np}, npos, poff, scr, st));
      SPX_TRY(summary_sync(P, st, &hs, {{poff + npos, 8}, {poff + multi_end, 8}}, tail + 2));
      if (hs.err & 4u) return fail(SPX_EUNSUPPORTED, "a row block is too dense for the LDS budget");
    }
  }
  P->nnz = tail[0];
  P->nzc = tail[1];
  P->nparts = tail[2];
  P->psplit = tail[3];
  P->nnz_tiny = (int64_t)hs.nnz_tiny;
  if (P->nparts > 0) {
    SPX_TRY(scr.get_n(P->nparts, &P->parts));
    k_parts<<<grid_for(npos, 256, (int64_t)cus * 16), 256, 0, st>>>(P->B, pc, pcs, P->list, npos, multi_begin, multi_end,
                                                                    P->gbm ? nbitmap : 0, P->cnt,
                                                                    P->off, blkcnt, nullptr, poff, P->parts,
                                                                    P->mults_d, nullptr, err);
    SPX_HIP(hipGetLastError());
    // bucket mode: range set-ups would outnumber multiplications 3 to 2
    // (building the lists costs about three walks over the cut columns' rows;
    // measured on R-MAT times tall-skinny B, the lists pay off above ~1.3)
    const int64_t nmulti = multi_end - multi_begin;
    const bool bucket_auto = tune.bucket_parts == 0 && hs.cut_mults > 0 && 2 * hs.setup > 3 * hs.cut_mults;
    if (P->psplit > 0 && (bucket_auto || tune.bucket_parts > 0) && nblk <= 4096 && nmulti * nblk <= (1ll << 27) &&
        B->nnz < (1ll << 31) && hs.cut_mults > 0) {
      int32_t* map = nullptr;
      unsigned *bcnt = nullptr, *bfill = nullptr;
      int64_t* boff = nullptr;
      SPX_TRY(scr.get_n(nmulti * nblk, &map));
      SPX_TRY(scr.get_n(P->psplit, &bcnt));
      SPX_TRY(scr.get_n(P->psplit, &bfill));
      SPX_TRY(scr.get_n(P->psplit + 1, &boff));
      SPX_TRY(scr.get_n((int64_t)hs.cut_mults, &P->qlist));  // a B entry reaches at most alen parts
      SPX_TRY(fill_u32(bcnt, P->psplit, 0, st));
      SPX_TRY(fill_u32(bfill, P->psplit, 0, st));
      k_bucket_map<<<grid_for(nmulti, 256, 4096), 256, 0, st>>>(pc, np, poff, multi_begin, multi_end, P->parts, map);
      SPX_HIP(hipGetLastError());
      const dim3 bgrid(64, (unsigned)std::min<int64_t>(nmulti, 4096));
      k_bucket<false><<<bgrid, 256, 0, st>>>(P->B, P->src, pc, P->list, np, poff, multi_begin, multi_end, P->parts,
                                              map, bcnt, nullptr, nullptr, nullptr, 0, err);
      SPX_HIP(hipGetLastError());
      SPX_TRY(exclusive_scan(LoadBucket{bcnt}, P->psplit, boff, scr, st));
      k_bucket<true><<<bgrid, 256, 0, st>>>(P->B, P->src, pc, P->list, np, poff, multi_begin, multi_end, P->parts,
                                             map, nullptr, boff, bfill, P->qlist, (int64_t)hs.cut_mults, err);
      SPX_HIP(hipGetLastError());
      k_bucket_parts<<<grid_for(nmulti, 256, 4096), 256, 0, st>>>(np, poff, multi_begin, multi_end, bcnt, boff,
                                                                  P->parts);
      SPX_HIP(hipGetLastError());
      SPX_TRY(summary_sync(P, st, &hs));
      if (hs.err & 32u) return fail(SPX_EDEVICE, "bucket lists exceeded their bound");
    }
    // work queues of the multi-part launch: one per row slice plus a
    // shared one (parts spanning all rows); the single-part launch has one
    P->nq_multi = pc.nslice + 1;
    SPX_TRY(scr.get_n(P->nq_multi + 1, &P->qoff_multi));
    SPX_TRY(scr.get_n(2, &P->qoff_single));
    SPX_TRY(scr.get_n(P->nq_multi + 2, &P->qctr));
    {
      const int64_t h[2] = {P->psplit, P->nparts};
      SPX_HIP(hipMemcpyAsync(P->qoff_single, h, sizeof(h), hipMemcpyHostToDevice, st));
    }
    if (P->psplit > 0 && pc.nslice <= 1) {
      // one queue with every multi part, the shared queue empty
      const int64_t h[3] = {0, P->psplit, P->psplit};
      SPX_HIP(hipMemcpyAsync(P->qoff_multi, h, sizeof(h), hipMemcpyHostToDevice, st));
    } else if (P->psplit > 0) {
      unsigned long long* hist = nullptr;
      Part* sorted = nullptr;
      SPX_TRY(scr.get_n(P->nq_multi + 1, &hist));
      SPX_TRY(scr.get_n(P->nparts, &sorted));
      SPX_TRY(fill_i64((int64_t*)hist, P->nq_multi + 1, 0, st));
      k_part_hist<<<grid_for(P->psplit, 256, 4096), 256, 0, st>>>(P->parts, P->psplit, hist);
      k_hist_offsets<<<1, 64, 0, st>>>(hist, P->nq_multi, 0, P->qoff_multi);
      k_part_scatter<<<grid_for(P->psplit, 256, 4096), 256, 0, st>>>(P->parts, P->psplit, hist, sorted);
      SPX_HIP(hipGetLastError());
      if (P->nparts > P->psplit)
        SPX_HIP(hipMemcpyAsync(sorted + P->psplit, P->parts + P->psplit, sizeof(Part) * (P->nparts - P->psplit),
                               hipMemcpyDeviceToDevice, st));
      P->parts = sorted;
    }
    if (P->psplit > 0) {
      k_parts_sum<<<grid_for(P->psplit, 256, 1024), 256, 0, st>>>(P->parts, P->psplit, &P->sum->nnz_multi);
      SPX_HIP(hipGetLastError());
      P->nnz_multi = -1;  // read by spx_plan_get_info
    }
  }
  P->mark(kEvPlan1, st);
  if (nnz_c) *nnz_c = P->nnz;
  if (nzc_c) *nzc_c = P->nzc;
  *plan = guard.release();
  return SPX_OK;
}

extern "C" int spx_spgemm_exec(spx_plan* plan, spx_mat* C) {
  if (!plan || plan->kind != kPlanGemm) return fail(SPX_EINVAL, "not a SpGEMM plan");
  auto* P = static_cast<GemmPlan*>(plan);
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  if (C->m != P->A.m || C->n != P->B.n) return fail(SPX_EINVAL, "C has the wrong dimensions");
  if (C->fmt != P->c_fmt) return fail(SPX_EINVAL, "C's format differs from the planned one");
  if (C->val_t != P->vt) return fail(SPX_EINVAL, "C's value type differs from the product's");
  if (C->ptr_t != SPX_PTR_I32 && C->ptr_t != SPX_PTR_I64) return fail(SPX_EINVAL, "bad C ptr_t");
  if (C->ptr_t == SPX_PTR_I32 && P->nnz >= (1ll << 31)) return fail(SPX_EOVERFLOW, "nnz(C) needs I64 pointers");
  if (!C->cp || (P->nnz > 0 && !C->ir) || (P->nnz > 0 && P->vt != SPX_VAL_BOOL && !C->num) ||
      (C->fmt == SPX_DCSC && P->nzc > 0 && !C->jc))
    return fail(SPX_EINVAL, "C buffers missing");
  C->nnz = P->nnz;
  C->nzc = C->fmt == SPX_DCSC ? P->nzc : 0;
  hipStream_t st = stream_of(&P->ctx);
  P->mark(kEvExec0, st);
  P->ran_parts = P->ran_tiny = false;
  if (P->nnz > 0) SPX_TRY(dispatch_numeric(P, C, st));
  else {
    P->mark(kEvMulti, st);
    P->mark(kEvParts, st);
    P->mark(kEvTiny, st);
  }
  if (C->fmt == SPX_CSC) {
    k_write_csc_cp<<<grid_for(C->n + 1, 256, 65536), 256, 0, st>>>(P->B, P->off, P->nslots, C->n, C->cp, C->ptr_t);
  } else if (P->nslots > 0) {
    k_write_dcsc<<<grid_for(P->nslots, 256, 65536), 256, 0, st>>>(P->B, P->cnt, P->off, P->zoff, P->nslots, C->jc,
                                                                   C->cp, C->ptr_t);
  } else {
    if (C->ptr_t == SPX_PTR_I64)
      SPX_TRY(fill_i64((int64_t*)C->cp, 1, 0, st));
    else
      SPX_TRY(fill_u32((uint32_t*)C->cp, 1, 0, st));
  }
  SPX_HIP(hipGetLastError());
  P->mark(kEvPtr, st);
  return SPX_OK;
}

extern "C" int spx_plan_get_times(spx_plan* plan, spx_times* times) {
  if (!plan || !times) return fail(SPX_EINVAL, "NULL argument");
  std::memset(times, 0, sizeof(*times));
  if (plan->kind == kPlanSum) plan = const_cast<spx_plan*>(sum_plan_inner(plan));
  if (plan->kind == kPlanContract) plan = const_cast<spx_plan*>(contract_plan_inner(plan));
  if (plan->kind != kPlanGemm) return fail(SPX_EINVAL, "not a SpGEMM plan");
  auto* P = static_cast<GemmPlan*>(plan);
  if (!P->profile) return fail(SPX_EINVAL, "plan was not created with ctx->profile set");
  SPX_HIP(hipEventSynchronize(P->ev[kEvPlan1]));
  SPX_HIP(hipEventElapsedTime(&times->symbolic_ms, P->ev[kEvPlan0], P->ev[kEvPlan1]));
  if (hipEventQuery(P->ev[kEvPtr]) == hipErrorNotReady) SPX_HIP(hipEventSynchronize(P->ev[kEvPtr]));
  float t = 0;
  if (hipEventElapsedTime(&t, P->ev[kEvExec0], P->ev[kEvPtr]) != hipSuccess) {
    (void)hipGetLastError();
    return SPX_OK;  // exec has not run
  }
  SPX_HIP(hipEventElapsedTime(&times->numeric_parts_ms, P->ev[kEvExec0], P->ev[kEvParts]));
  SPX_HIP(hipEventElapsedTime(&times->numeric_multi_ms, P->ev[kEvExec0], P->ev[kEvMulti]));
  SPX_HIP(hipEventElapsedTime(&times->numeric_tiny_ms, P->ev[kEvParts], P->ev[kEvTiny]));
  SPX_HIP(hipEventElapsedTime(&times->pointers_ms, P->ev[kEvTiny], P->ev[kEvPtr]));
  return SPX_OK;
}

extern "C" int spx_plan_get_info(const spx_plan* plan, spx_plan_info* info) {
  if (!plan || !info) return fail(SPX_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  if (plan->kind == kPlanSum) plan = sum_plan_inner(plan);
  if (plan->kind == kPlanContract) plan = contract_plan_inner(plan);
  if (plan->kind != kPlanGemm) return SPX_OK;
  auto* P = const_cast<GemmPlan*>(static_cast<const GemmPlan*>(plan));
  if (P->nnz_multi < 0) {
    int64_t v = 0;
    SPX_TRY(read_device_words(stream_of(&P->ctx), {{&P->sum->nnz_multi, 8}}, &v));
    P->nnz_multi = v;
  }
  const int64_t* bo = P->binoff_h;
  info->mults = P->mults;
  info->nnz = P->nnz;
  info->nzc = P->nzc;
  info->cols_empty = bo[kBinEmpty + 1] - bo[kBinEmpty];
  info->cols_tiny = bo[kBinTiny + 1] - bo[kBinTiny];
  info->cols_medium = bo[kBinTiny] - bo[kBinHash0];
  info->cols_heavy = bo[kBinHash0] - bo[0];
  info->heavy_parts = P->nparts;
  info->nnz_tiny = P->nnz_tiny;
  info->nnz_multi = P->nnz_multi;
  info->multi_parts = P->psplit;
  return SPX_OK;
}

extern "C" void spx_plan_destroy(spx_plan* plan) { delete plan; }

const int64_t* spx::gemm_plan_offsets(const spx_plan* plan) {
  if (!plan || plan->kind != kPlanGemm) return nullptr;
  return static_cast<const GemmPlan*>(plan)->off;
}

extern "C" int spx_spgemm(const spx_ctx* ctx, const spx_mat* A, const spx_mat* B, int32_t semiring, int32_t c_fmt,
                          spx_mat* C) {
  if (!C) return fail(SPX_EINVAL, "C is NULL");
  spx_plan* plan = nullptr;
  int64_t nnz = 0, nzc = 0;
  SPX_TRY(spx_spgemm_plan(ctx, A, B, semiring, c_fmt, nullptr, &plan, &nnz, &nzc));
  std::unique_ptr<spx_plan> guard(plan);
  auto* P = static_cast<GemmPlan*>(plan);
  OutAlloc oa(ctx);
  spx_mat out{};
  out.m = A->m;
  out.n = B->n;
  out.fmt = c_fmt;
  out.ptr_t = SPX_PTR_I64;
  out.val_t = P->vt;
  const int64_t ncp = (c_fmt == SPX_CSC ? B->n : nzc) + 1;
  SPX_TRY(oa.get((size_t)ncp * 8, &out.cp));
  SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz, 1) * 4, reinterpret_cast<void**>(&out.ir)));
  if (P->vt != SPX_VAL_BOOL) SPX_TRY(oa.get((size_t)std::max<int64_t>(nnz, 1) * value_size(P->vt), &out.num));
  if (c_fmt == SPX_DCSC) SPX_TRY(oa.get((size_t)std::max<int64_t>(nzc, 1) * 4, reinterpret_cast<void**>(&out.jc)));
  SPX_TRY(spx_spgemm_exec(plan, &out));
  oa.keep();
  *C = out;
  return SPX_OK;
}
